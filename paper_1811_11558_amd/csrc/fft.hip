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

// Complex elements of one block's LDS tile in the row kernels, chosen per
// kernel and precision by measurement on 256^2 x 64: a smaller tile lets
// more blocks share a CU (the forward transform gains: 16 KiB), a larger one
// gives the inverse transform's strided reads longer runs (32 KiB in
// float64; 16 KiB in float32).
template <typename T>
__host__ __device__ constexpr int r2c_tile_elems() { return sizeof(T) == 8 ? 1024 : 2048; }
template <typename T>
__host__ __device__ constexpr int c2r_tile_elems() { return 2048; }
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
__host__ __device__ constexpr int r2c_seq(int n) { return row_seq(n, (int)sizeof(cpx<T>), r2c_tile_elems<T>()); }
template <typename T>
__host__ __device__ constexpr int c2r_seq(int n) { return row_seq(n, (int)sizeof(cpx<T>), c2r_tile_elems<T>()); }
// Columns (planes) per block of the column (y) kernels.  The mode-major side
// S[kx][ky][p] is touched in runs of B consecutive planes, so B is the 32 KiB
// tile's share unless that makes runs shorter than 64 bytes (ny >= 1024 in
// float64, >= 1024 in float32), in which case the tile grows up to the
// 160 KiB of LDS a block may use (powers of two).  Measured: 32-byte runs ran
// at 1.5 TB/s, 64-byte runs at 4.4 TB/s, and 64 KiB tiles with 256-byte runs
// were slower than 32 KiB ones at ny = 256.
__host__ __device__ constexpr int col_batch_bytes(int n, int csize) {
  int b = (32768 / csize) / n;
  if (b < 1) b = 1;
  const int minb = 64 / csize;
  int maxb = 1;
  while (2 * maxb * (n + 1) * csize <= 160 * 1024) maxb *= 2;
  if (b < minb) b = minb < maxb ? minb : maxb;
  return b;
}
template <typename T>
__host__ __device__ constexpr int col_batch(int n) { return col_batch_bytes(n, (int)sizeof(cpx<T>)); }

// NB transforms of length N = 2^LOGN held at buf[b * ld + k] (NB <= NBMAX),
// Stockham autosort: one radix-2 stage first when LOGN is odd, then radix-4
// stages.  All index arithmetic is shifts and masks.  Called by all NT threads.
template <typename T, int LOGN, int NBMAX, bool INV>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, int ld, int NB, const cpx<T>* __restrict__ tw) {
  constexpr int N = 1 << LOGN;
  const int tid = threadIdx.x;
  if constexpr (LOGN & 1) {
    constexpr int H = N / 2;
    constexpr int MB = (NBMAX * H + NT - 1) / NT;
    const int nb = NB * H;
    cpx<T> v0[MB], v1[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      int j = tid + u * NT;
      if (j < nb) {
        int b = j >> (LOGN - 1), jj = j & (H - 1);
        v0[u] = buf[b * ld + jj];
        v1[u] = buf[b * ld + jj + H];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      int j = tid + u * NT;
      if (j < nb) {
        int b = j >> (LOGN - 1), jj = j & (H - 1);
        buf[b * ld + 2 * jj] = add(v0[u], v1[u]);
        buf[b * ld + 2 * jj + 1] = sub(v0[u], v1[u]);
      }
    }
    __syncthreads();
  }
  constexpr int Q = N / 4;
  constexpr int MB4 = (NBMAX * Q + NT - 1) / NT;
  const int nb4 = NB * Q;
#pragma unroll
  for (int ls = (LOGN & 1); ls < LOGN; ls += 2) {
    const int ns = 1 << ls;
    const int tstep = N >> (ls + 2);
    cpx<T> v[MB4][4];
#pragma unroll
    for (int u = 0; u < MB4; ++u) {
      int j = tid + u * NT;
      if (j < nb4) {
        int b = j >> (LOGN - 2), jj = j & (Q - 1);
        const cpx<T>* src = buf + b * ld + jj;
        v[u][0] = src[0];
        v[u][1] = src[Q];
        v[u][2] = src[2 * Q];
        v[u][3] = src[3 * Q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MB4; ++u) {
      int j = tid + u * NT;
      if (j < nb4) {
        int b = j >> (LOGN - 2), jj = j & (Q - 1);
        int k = jj & (ns - 1);
        cpx<T> a0 = v[u][0];
        cpx<T> a1 = v[u][1], a2 = v[u][2], a3 = v[u][3];
        if (ls > 0) {
          a1 = mul(a1, twid<T, INV>(tw, k * tstep));
          a2 = mul(a2, twid<T, INV>(tw, 2 * k * tstep));
          a3 = mul(a3, twid<T, INV>(tw, 3 * k * tstep));
        }
        cpx<T> s02 = add(a0, a2), d02 = sub(a0, a2);
        cpx<T> s13 = add(a1, a3), d13 = sub(a1, a3);
        // forward: y1 = d02 - i d13, y3 = d02 + i d13 (conjugate for inverse)
        cpx<T> id13 = INV ? mul_i(d13) : mul_mi(d13);
        int o = b * ld + ((jj >> ls) << (ls + 2)) + k;
        buf[o] = add(s02, s13);
        buf[o + ns] = add(d02, id13);
        buf[o + 2 * ns] = sub(s02, s13);
        buf[o + 3 * ns] = sub(d02, id13);
      }
    }
    __syncthreads();
  }
}

// Rows of nx = 2^LOGN reals -> half spectra.  Block = R consecutive rows of
// one plane (R even, R | ny), two rows per complex sequence.  Output
// X[(plane * kxh + k) * ny + y].
// If bsum is not NULL, block b also writes the float64 sum of its R rows to
// bsum[b] (the plane means of the mean mode are then formed in float64).
template <typename T, int LOGN, bool NTL>
__global__ __launch_bounds__(NT) void k_x_r2c(InSegments seg, cpx<T>* __restrict__ out, int ny, int R,
                                             const cpx<T>* __restrict__ tw, double* __restrict__ bsum,
                                             LayerSkip skip) {
  constexpr int N = 1 << LOGN;
  constexpr int SEQ = r2c_seq<T>(N);
  constexpr int ld = N + 1;
  constexpr int kxh = N / 2 + 1;
  __shared__ cpx<T> buf[SEQ * ld];
  const size_t row0 = (size_t)blockIdx.x * R;
  const size_t plane = row0 / ny;
  const int y0 = (int)(row0 - plane * ny);
  // a layer without plastic strain: its rows sum to zero, nothing to transform
  if (skip.zact && (int)plane < skip.nw && (int)(plane % skip.nz) >= *skip.zact) {
    if (bsum && threadIdx.x == 0) bsum[blockIdx.x] = 0.0;
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
    __shared__ double red[NT];
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < MV; ++u) {
      int i = threadIdx.x + u * NT;
      if (i < tot) acc += v[u].x + v[u].y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
  }
  __syncthreads();
  lds_fft<T, LOGN, SEQ, false>(buf, ld, R / 2, tw);
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
template <typename T, int LOGN, bool NTL>
__global__ __launch_bounds__(NT) void k_y_fwd(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int kxh,
                                             int NP, int ldp, const cpx<T>* __restrict__ tw, LayerSkip skip) {
  constexpr int N = 1 << LOGN;
  constexpr int B = col_batch<T>(N);
  static_assert((B * N) % NT == 0, "tile must be a multiple of the block");
  constexpr int ld = N + 1;
  __shared__ cpx<T> buf[B * ld];
  const int npb = (NP + B - 1) / B;
  const int lb = xcd_block();
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
  lds_fft<T, LOGN, B, false>(buf, ld, nb, tw);
  // consecutive lanes take consecutive planes of one ky: runs of nb elements
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = threadIdx.x + u * NT;
    const int ky = i / B, b = i - ky * B;
    if (b < nb) out[((size_t)kx * N + ky) * ldp + p0 + b] = buf[b * ld + ky];
  }
}

// Inverse column transform: S[kx][ky][p] -> X[p][kx][y].
template <typename T, int LOGN, bool NTL>
__global__ __launch_bounds__(NT) void k_y_inv(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int kxh,
                                             int NP, int ldp, const cpx<T>* __restrict__ tw) {
  constexpr int N = 1 << LOGN;
  constexpr int B = col_batch<T>(N);
  constexpr int ld = N + 1;
  __shared__ cpx<T> buf[B * ld];
  const int npb = (NP + B - 1) / B;
  const int lb = xcd_block();
  const int kx = lb / npb;
  const int p0 = (lb - kx * npb) * B;
  const int nb = min(B, NP - p0);
  static_assert((B * N) % NT == 0, "tile must be a multiple of the block");
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
  lds_fft<T, LOGN, B, true>(buf, ld, nb, tw);
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
// of that plane (the mean mode computed in float64).
// NTS: the outputs (without the epilogue) are stored as streaming writes.
template <typename T, int LOGN, bool NTS>
__global__ __launch_bounds__(NT) void k_x_c2r(const cpx<T>* __restrict__ in, OutSegments seg, int ny, int R,
                                             double scale, const cpx<T>* __restrict__ tw,
                                             const double* __restrict__ padd, ResidEpilogue ep) {
  constexpr int N = 1 << LOGN;
  constexpr int SEQ = c2r_seq<T>(N);
  constexpr int ld = N + 1;
  constexpr int kxh = N / 2 + 1;
  constexpr int nyq = N / 2;
  __shared__ cpx<T> buf[SEQ * ld];
  const size_t row0 = (size_t)blockIdx.x * R;
  const int plane = (int)(row0 / ny);
  const int y0 = (int)(row0 - (size_t)plane * ny);
  const int hp = R / 2;                  // a power of two (R = ny or 2 SEQ)
  const int lhp = __builtin_ctz(hp);
  const int tot = kxh * hp;
  // all loads first (slots past the end repeat the last pair, which writes
  // the same values again), then the LDS writes
  constexpr int MV = (kxh * SEQ + NT - 1) / NT;
  cpx<T> v0[MV], v1[MV];
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = min((int)threadIdx.x + u * NT, tot - 1);
    const int k = i >> lhp, pr = i - (k << lhp);
    const size_t a = ((size_t)plane * kxh + k) * ny + y0 + 2 * pr;
    v0[u] = in[a];
    v1[u] = in[a + 1];
  }
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = min((int)threadIdx.x + u * NT, tot - 1);
    const int k = i >> lhp, pr = i - (k << lhp);
    const cpx<T> X0 = v0[u], X1 = v1[u];
    if (k == 0 || k == nyq) {
      buf[pr * ld + k] = mk(X0.x, X1.x);
    } else {
      buf[pr * ld + k] = mk(X0.x - X1.y, X0.y + X1.x);
      buf[pr * ld + N - k] = mk(X0.x + X1.y, X1.x - X0.y);
    }
  }
  __syncthreads();
  lds_fft<T, LOGN, SEQ, true>(buf, ld, hp, tw);
  int s = 0;
  while (s + 1 < seg.n && plane >= seg.first[s + 1]) ++s;
  double* dst = seg.ptr[s] + ((size_t)(plane - seg.first[s]) * ny + y0) * N;
  const double add = padd ? padd[plane] : 0.0;
  const int tot2 = R * N / 2;
  double2* d2 = reinterpret_cast<double2*>(dst);
  if (!ep.x) {
    // The operator's outputs are not read again by the operator, so they
    // are stored as streaming (non-temporal) writes, which do not displace
    // the spectrum buffers from the last-level cache.  Measured at
    // 256^2 x 64 float64: this kernel 92.8 -> 71.7 us, the whole
    // application 0.427 -> 0.421 ms (the column transforms, whose buffers
    // the cache then holds differently, lose part of the gain).  The
    // contact solver's compliance, read at once by the next kernel, keeps
    // ordinary stores.
    typedef double v2d __attribute__((ext_vector_type(2)));
    for (int i = threadIdx.x; i < tot2; i += NT) {
      int r = (2 * i) >> LOGN, x = (2 * i) & (N - 1);
      const cpx<T>* b = buf + (r >> 1) * ld + x;
      v2d o;
      if (r & 1) { o.x = (double)b[0].y * scale + add; o.y = (double)b[1].y * scale + add; }
      else { o.x = (double)b[0].x * scale + add; o.y = (double)b[1].x * scale + add; }
      if constexpr (NTS) __builtin_nontemporal_store(o, reinterpret_cast<v2d*>(d2 + i));
      else *reinterpret_cast<v2d*>(d2 + i) = o;
    }
    return;
  }
  // residual epilogue (the residual is the first and only segment)
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
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_down(s0, o, 64);
    s1 += __shfl_down(s1, o, 64);
  }
  __shared__ double red[2][NT / 64];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s0;
    red[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      a += red[0][w];
      c += red[1][w];
    }
    const int cp = plane / ep.nz, z = plane - cp * ep.nz;
    const double wt = (cp < 3 ? 1.0 : 2.0) * (ep.wz ? ep.wz[z] : ((z == 0 || z == ep.nz - 1) ? 0.5 : 1.0));
    ep.part[2 * blockIdx.x] = wt * a;
    ep.part[2 * blockIdx.x + 1] = wt * c;
  }
}

// R of a row kernel launch: 2 SEQ rows, or the whole plane when it is shorter
int rows_per_block(int seq, int ny) { return 2 * seq < ny ? 2 * seq : ny; }

template <typename T>
int cols_per_block(int ny) {
  return col_batch<T>(ny);
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

int ilog2(int n) { return 31 - __builtin_clz((unsigned)n); }

}  // namespace

template <typename T>
int x_r2c_blocks_per_plane(int nx, int ny) {
  return ny / rows_per_block(r2c_seq<T>(nx), ny);
}

template <typename T>
hipError_t launch_x_r2c(const InSegments& seg, cpx<T>* out, int nx, int ny, size_t nplanes, const cpx<T>* tw,
                        hipStream_t st, double* bsum, bool stream_in, const LayerSkip& skip) {
  if (seg.n < 1 || seg.n > 2 || seg.first[0] != 0) return hipErrorInvalidValue;
  int R = rows_per_block(r2c_seq<T>(nx), ny);
  dim3 grid((unsigned)(nplanes * (size_t)ny / R));
#define CALL(L)                                                                                        \
  if (stream_in) hipLaunchKernelGGL((k_x_r2c<T, L, true>), grid, dim3(NT), 0, st, seg, out, ny, R, tw, bsum, skip); \
  else hipLaunchKernelGGL((k_x_r2c<T, L, false>), grid, dim3(NT), 0, st, seg, out, ny, R, tw, bsum, skip)
  FVIM_LOGN_SWITCH(ilog2(nx), CALL)
#undef CALL
  return hipGetLastError();
}

template <typename T>
hipError_t launch_x_r2c(const double* in, cpx<T>* out, int nx, int ny, size_t nplanes, const cpx<T>* tw,
                        hipStream_t st, double* bsum, bool stream_in) {
  InSegments seg;
  seg.n = 1;
  seg.first[0] = seg.first[1] = 0;
  seg.ptr[0] = seg.ptr[1] = in;
  return launch_x_r2c<T>(seg, out, nx, ny, nplanes, tw, st, bsum, stream_in, LayerSkip{});
}

template <typename T>
hipError_t launch_y_fwd(const cpx<T>* in, cpx<T>* out, int ny, int kxh, int NP, int ldp, const cpx<T>* tw,
                        hipStream_t st, bool stream_in, const LayerSkip& skip) {
  if (ldp < NP) return hipErrorInvalidValue;
  int B = cols_per_block<T>(ny);
  dim3 grid((unsigned)(kxh * ((NP + B - 1) / B)));
#define CALL(L)                                                                                       \
  if (stream_in) hipLaunchKernelGGL((k_y_fwd<T, L, true>), grid, dim3(NT), 0, st, in, out, kxh, NP, ldp, tw, skip); \
  else hipLaunchKernelGGL((k_y_fwd<T, L, false>), grid, dim3(NT), 0, st, in, out, kxh, NP, ldp, tw, skip)
  FVIM_LOGN_SWITCH(ilog2(ny), CALL)
#undef CALL
  return hipGetLastError();
}

template <typename T>
hipError_t launch_y_inv(const cpx<T>* in, cpx<T>* out, int ny, int kxh, int NP, int ldp, const cpx<T>* tw,
                        hipStream_t st, bool stream_in) {
  if (ldp < NP) return hipErrorInvalidValue;
  int B = cols_per_block<T>(ny);
  dim3 grid((unsigned)(kxh * ((NP + B - 1) / B)));
#define CALL(L)                                                                                       \
  if (stream_in) hipLaunchKernelGGL((k_y_inv<T, L, true>), grid, dim3(NT), 0, st, in, out, kxh, NP, ldp, tw); \
  else hipLaunchKernelGGL((k_y_inv<T, L, false>), grid, dim3(NT), 0, st, in, out, kxh, NP, ldp, tw)
  FVIM_LOGN_SWITCH(ilog2(ny), CALL)
#undef CALL
  return hipGetLastError();
}

template <typename T>
hipError_t launch_x_c2r(const cpx<T>* in, const OutSegments& seg, int nx, int ny, size_t nplanes,
                        double scale, const cpx<T>* tw, hipStream_t st, const double* padd,
                        const ResidEpilogue& ep, bool stream_out) {
  // the epilogue reads its fields at the output's own offsets: one segment
  // holding the 6 nz strain planes from plane 0
  if (ep.x && (seg.n != 1 || seg.first[0] != 0 || !ep.part || ep.nz < 1 || nplanes != (size_t)6 * ep.nz))
    return hipErrorInvalidValue;
  int R = rows_per_block(c2r_seq<T>(nx), ny);
  dim3 grid((unsigned)(nplanes * (size_t)ny / R));
#define CALL(L)                                                                                          \
  if (stream_out) hipLaunchKernelGGL((k_x_c2r<T, L, true>), grid, dim3(NT), 0, st, in, seg, ny, R, scale, tw, padd, ep); \
  else hipLaunchKernelGGL((k_x_c2r<T, L, false>), grid, dim3(NT), 0, st, in, seg, ny, R, scale, tw, padd, ep)
  FVIM_LOGN_SWITCH(ilog2(nx), CALL)
#undef CALL
  return hipGetLastError();
}

template <typename T>
int x_c2r_blocks(int nx, int ny, size_t nplanes) {
  return (int)(nplanes * (size_t)ny / rows_per_block(c2r_seq<T>(nx), ny));
}
template int x_c2r_blocks<double>(int, int, size_t);
template int x_c2r_blocks<float>(int, int, size_t);

template hipError_t launch_x_r2c<double>(const double*, cpx<double>*, int, int, size_t, const cpx<double>*,
                                         hipStream_t, double*, bool);
template hipError_t launch_x_r2c<double>(const InSegments&, cpx<double>*, int, int, size_t,
                                         const cpx<double>*, hipStream_t, double*, bool, const LayerSkip&);
template hipError_t launch_x_r2c<float>(const InSegments&, cpx<float>*, int, int, size_t, const cpx<float>*,
                                        hipStream_t, double*, bool, const LayerSkip&);
template hipError_t launch_x_r2c<float>(const double*, cpx<float>*, int, int, size_t, const cpx<float>*,
                                        hipStream_t, double*, bool);
template int x_r2c_blocks_per_plane<double>(int, int);
template int x_r2c_blocks_per_plane<float>(int, int);
template hipError_t launch_y_fwd<double>(const cpx<double>*, cpx<double>*, int, int, int, int,
                                         const cpx<double>*, hipStream_t, bool, const LayerSkip&);
template hipError_t launch_y_fwd<float>(const cpx<float>*, cpx<float>*, int, int, int, int, const cpx<float>*,
                                        hipStream_t, bool, const LayerSkip&);
template hipError_t launch_y_inv<double>(const cpx<double>*, cpx<double>*, int, int, int, int,
                                         const cpx<double>*, hipStream_t, bool);
template hipError_t launch_y_inv<float>(const cpx<float>*, cpx<float>*, int, int, int, int, const cpx<float>*,
                                        hipStream_t, bool);
template hipError_t launch_x_c2r<double>(const cpx<double>*, const OutSegments&, int, int, size_t, double,
                                         const cpx<double>*, hipStream_t, const double*,
                                         const ResidEpilogue&, bool);
template hipError_t launch_x_c2r<float>(const cpx<float>*, const OutSegments&, int, int, size_t, double,
                                        const cpx<float>*, hipStream_t, const double*,
                                         const ResidEpilogue&, bool);

}  // namespace fvim
