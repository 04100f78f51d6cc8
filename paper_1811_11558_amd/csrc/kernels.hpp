// Launch wrappers shared between the translation units of the library.
#pragma once
#include "common.hpp"

namespace fvim {

// Destination of the planes leaving the inverse x transform: plane p goes to
// ptr[s] at local plane p - first[s] for the last s with first[s] <= p.
struct OutSegments {
  int n;
  int first[4];
  double* ptr[4];
};

// Source of the planes entering the forward x transform: plane p comes from
// ptr[s] at local plane p - first[s] for the last s with first[s] <= p.
struct InSegments {
  int n;
  int first[2];
  const double* ptr[2];
};

// Depth layers without plastic strain: with zact set, eigenstrain plane p
// (p < nw = 6 nz, depth p % nz) is known to be zero when p % nz >= *zact
// (a device value), and the forward transforms skip it (its spectrum is then
// not written; the depth pass reads only layers below *zact).
struct LayerSkip {
  const int* zact;
  int nz, nw;
};
// Launch choice of a transform kernel: the LDS tile (0: half the default,
// 1: the default, 2: twice) and the radix of the Stockham stages (4 or 8).
// Only lengths 2^FFT_TUNE_MIN_LOGN .. 2^FFT_TUNE_MAX_LOGN have the
// alternatives; fft_effective gives what a launch of length 2^logn runs.
struct FftChoice {
  int tile = 1;
  int radix = 4;
};
constexpr int FFT_TUNE_MIN_LOGN = 5, FFT_TUNE_MAX_LOGN = 10;
FftChoice fft_effective(int logn, FftChoice ch);

// bsum (optional): float64 sum of the rows of each block, blocks of a plane
// consecutive (x_r2c_blocks_per_plane of them).  stream_in: the launch reads
// its input for the last time with streaming (non-temporal) loads (see
// operator_streaming); every launcher below takes the same flag.
template <typename T>
hipError_t launch_x_r2c(const InSegments& seg, cpx<T>* out, int nx, int ny, size_t nplanes, const cpx<T>* tw,
                        hipStream_t st, double* bsum = nullptr, bool stream_in = false,
                        const LayerSkip& skip = LayerSkip{}, FftChoice ch = FftChoice{});
template <typename T>
hipError_t launch_x_r2c(const double* in, cpx<T>* out, int nx, int ny, size_t nplanes, const cpx<T>* tw,
                        hipStream_t st, double* bsum = nullptr, bool stream_in = false);
template <typename T>
int x_r2c_blocks_per_plane(int nx, int ny, FftChoice ch = FftChoice{});
// the most blocks per plane any choice gives (buffers sized for tuning)
template <typename T>
int x_r2c_max_blocks_per_plane(int nx, int ny);
// Column transforms between X[p][kx][y] (p < NP) and the mode-major
// S[kx][ky][ldp] (record stride ldp >= NP; the padding is not touched).
template <typename T>
hipError_t launch_y_fwd(const cpx<T>* in, cpx<T>* out, int ny, int kxh, int NP, int ldp, const cpx<T>* tw,
                        hipStream_t st, bool stream_in = false, const LayerSkip& skip = LayerSkip{},
                        FftChoice ch = FftChoice{});
template <typename T>
hipError_t launch_y_inv(const cpx<T>* in, cpx<T>* out, int ny, int kxh, int NP, int ldp, const cpx<T>* tw,
                        hipStream_t st, bool stream_in = false, FftChoice ch = FftChoice{});
// Record stride of a mode-major spectrum of np planes: a whole number of
// 128-byte lines, so every mode's record starts on a line.
template <typename T>
inline int mode_stride(int np) {
  const int q = 128 / (int)sizeof(cpx<T>);
  return (np + q - 1) / q * q;
}
// Residual epilogue of the inverse x transform (plasticity iteration): with
// x set, each output value w of the first segment (the 6 nz strain planes)
// is replaced by r = x - w, and block b writes wt sum r.r to part[2 b] and,
// with Fo, wt sum Fo.(r - Fo) to part[2 b + 1]; wt = 2 for shear planes
// (plane / nz >= 3) times the depth weight of the plane's node: wz[z] if
// given (device, nz), else 1/2 at the first and last node and 1 between.
struct ResidEpilogue {
  const double* x;
  const double* Fo;
  double* part;
  int nz;
  const double* wz;
};
// padd (optional): float64 constant added to each plane of the output.  No
// streaming loads here: keeping its input cached measured faster (the next
// application's y_inv writes the same buffer).  stream_out: the outputs
// (without the epilogue) are stored as streaming writes.
template <typename T>
hipError_t launch_x_c2r(const cpx<T>* in, const OutSegments& seg, int nx, int ny, size_t nplanes,
                        double scale, const cpx<T>* tw, hipStream_t st, const double* padd = nullptr,
                        const ResidEpilogue& ep = ResidEpilogue{}, bool stream_out = false,
                        FftChoice ch = FftChoice{});
// blocks of a launch_x_c2r over nplanes planes (partial-sum pairs it writes)
template <typename T>
int x_c2r_blocks(int nx, int ny, size_t nplanes, FftChoice ch = FftChoice{});
template <typename T>
int x_c2r_max_blocks(int nx, int ny, size_t nplanes);

// One launch of a transform kernel over several grids (up to
// XFORM_BATCH_MAX, lengths up to 2^XFORM_BATCH_MAX_LOGN), each with the
// default choice of its length: the grids' parameters travel as the kernel
// argument.  logn: log2 of the kernel's transform length (nx for the row
// kernels, ny for the column kernels); NP: planes (row kernels: planes of
// ny rows; column kernels: planes NP with record stride ldp); R and first
// are filled by launch_xform_batch.  Row kernels use ny, iseg / oseg, tw,
// bsum (x_r2c, may be NULL), padd and nts (x_c2r); column kernels use in,
// out, kxh, NP, ldp, tw.
constexpr int XFORM_BATCH_MAX = 8, XFORM_BATCH_MAX_LOGN = 9;
struct XformBatch {
  int n;
  int first[XFORM_BATCH_MAX + 1];
  int logn[XFORM_BATCH_MAX];
  int ny[XFORM_BATCH_MAX], R[XFORM_BATCH_MAX], NP[XFORM_BATCH_MAX];
  int kxh[XFORM_BATCH_MAX], ldp[XFORM_BATCH_MAX], nts[XFORM_BATCH_MAX];
  const void* in[XFORM_BATCH_MAX];
  void* out[XFORM_BATCH_MAX];
  const void* tw[XFORM_BATCH_MAX];
  double* bsum[XFORM_BATCH_MAX];
  const double* padd[XFORM_BATCH_MAX];
  InSegments iseg[XFORM_BATCH_MAX];
  OutSegments oseg[XFORM_BATCH_MAX];
};
// kind: 0 x_r2c, 1 y_fwd, 2 y_inv, 3 x_c2r
template <typename T>
hipError_t launch_xform_batch(int kind, XformBatch& b, hipStream_t st);
// Fills b.R and b.first of a batched transform (as launch_xform_batch does)
// and returns the dynamic LDS bytes it needs (0 for an invalid table).
template <typename T>
size_t xform_batch_prepare(int kind, XformBatch& b);
template <typename T>
int x_r2c_batch_blocks_per_plane(int nx, int ny);

// Per-mode depth pass.  Input spectra (unnormalised DFTs) in mode-major
// layout in[mode][ld_in]: the plastic strain as [6][nz] at offset 0 (if
// has_w) and the traction as [3] at offset off_t (if has_t); output
// out[mode][ld_out] holding the np_out requested planes at
// plane offsets off_* (negative = not requested): strain and stress as
// [6][nz], displacement as [3][nz], surface u3 as one plane.
struct DepthParams {
  int nx, ny, nz, kxh;
  double lx, ly, h;       // in-plane domain lengths, depth-node spacing
  double mu, kappa;       // shear modulus, lambda / mu
  double norm;            // 1 / (nx ny)
  int has_w, has_t, k0_include;
  int k0_external;        // 1: the mean mode is added by the caller in float64; write 0 here
  int np_in, off_t, ld_in;
  int np_out, ld_out;
  int off_strain, off_stress, off_disp, off_u3;
  const void* mtab;       // ModeConst<T>[kxh * ny] of this grid (launch_mode_table)
  // Nyquist modes: NULL -> a second launch averages each mode's 2 or 4 sign
  // replicas in turn; else the main launch evaluates every replica as a
  // mode of its own into depth_replicas(ny, kxh) records of stride ld_out
  // here, and the second launch averages them
  void* rep_out;
  int nt_in;              // the main launch reads the input with streaming loads
  const int* zact;        // if set: eigenstrain layers z >= *zact are zero and not read
  const double* hz;       // if set (device, nz - 1): non-uniform element lengths
                          // z_(e+1) - z_e; h and the mode table's s, r, G0..H0p
                          // are then unused.  Not in batched launches
  // ratios of kappa, filled by launch_depth: 1/(kappa+2), (kappa+1)/(kappa+2),
  // 1/(2(kappa+2)), kappa/(kappa+2), (kappa+2)/(2(kappa+1)), 1/(2 kappa+2)
  double ikp2, kk, i2k4, kapkp2, cfac, ik2;
};

// Constants of one in-plane mode for the depth pass, computed once per grid
// in float64 and stored in the working precision: s = |q| h, r = exp(-s),
// the element functions G0, G0', H0, H0' of s, and 1/|q| (all 0 for the
// mean mode).
template <typename T>
struct alignas(16) ModeConst {
  T s, r, G0, G0p, H0, H0p, iq, pad;
};

// Depth pass over several grids in one launch per part: the host table lists
// each grid's parameters (derived constants filled by depth_derive, rep_out
// set: the Nyquist sign replicas are modes of the main launch), input and
// output spectra, and prefix counts of blocks: first_main for the main launch
// (modes and replicas, depth_groups_per_block(cfg) per block), first_nyq for
// the averaging launch (one block per Nyquist mode).  dtab is a device copy
// target.  Every grid must request the same kinds of output and have nz <=
// the configuration's capacity.
constexpr int DEPTH_BATCH_MAX = 8;
struct DepthBatch {
  int n;
  int first_main[DEPTH_BATCH_MAX + 1];
  int first_nyq[DEPTH_BATCH_MAX + 1];
  DepthParams prm[DEPTH_BATCH_MAX];
  const void* in[DEPTH_BATCH_MAX];
  void* out[DEPTH_BATCH_MAX];
};
void depth_derive(DepthParams& p);

// The whole fused operator application over several grids: the four
// batched transform tables (x_r2c, y_fwd, y_inv, x_c2r) and the depth table.
struct OpBatch {
  XformBatch x[4];
  DepthBatch d;
};
// One cooperative launch runs every stage of the batched application, the
// blocks looping over each stage's blocks and meeting at a grid barrier
// between stages (float64, strain output only, depth configurations of
// nz <= 128).  dev: device copy of the table (sizeof(OpBatch)).  Returns
// hipErrorNotSupported when the batch does not qualify.
template <typename T>
hipError_t launch_operator_persistent(OpBatch& host, OpBatch* dev, int depth_cfg, bool disp, bool wx,
                                      hipStream_t st);
// Sign replicas of the Nyquist modes: 2 for each of the ny + kxh - 1 modes on
// the kx = nx/2 column or the ky = ny/2 row, 2 more for the corner.
inline int depth_replicas(int ny, int kxh) { return 2 * (ny + kxh); }
int depth_groups_per_block(int cfg);
template <typename T>
hipError_t launch_depth_batch(const DepthBatch& host, DepthBatch* dtab, int cfg, hipStream_t st);

template <typename T>
hipError_t launch_mode_table(ModeConst<T>* tab, int nx, int ny, double lx, double ly, double h, hipStream_t st);

// part: 0 = every mode (two launches), 1 = all but the Nyquist modes,
// 2 = the Nyquist modes only.
template <typename T>
hipError_t launch_depth(const cpx<T>* in, cpx<T>* out, const DepthParams& p, int cfg, hipStream_t st,
                        int part = 0);
int depth_num_configs();
bool depth_config_valid(int id, int nz);
int depth_default_config(int nz);

// Mean-mode (k = 0) fields in float64 from the block sums of the input
// planes: out[plane] for every output plane (strain, stress, displacement,
// surface u3 segments as in DepthParams).
hipError_t launch_k0_fields(const double* wsum, int wblocks, const double* tsum, int tblocks, double* out,
                            const DepthParams& p, hipStream_t st);

// Pointwise kernels (float64).
hipError_t launch_return_map(const double* d_eps, const double* sig_n, const double* ep_n, double* d_eps_p,
                             double* d_ep, double* sig_np1, size_t nvox, double lam, double mu,
                             double sy0, double eh, hipStream_t st);
// Return map at the trial point x + cf F (F may be NULL: at x); the trial
// point is stored in xt when F and xt are given; writes d_eps_p only.  With
// layer_flags, layer_flags[z] is set to 1 for every depth layer z (voxel v
// in layer v >> lp) where d_eps_p is not zero (the caller clears them).
// With zwrite (device), d_eps_p is known to hold zeros in the layers >=
// *zwrite, and elastic voxels there are not stored again.
hipError_t launch_trial_return_map(const double* x, const double* F, double cf, double* xt, const double* sig_n,
                                   const double* ep_n, double* d_eps_p, size_t nvox, double lam, double mu,
                                   double sy0, double eh, hipStream_t st, int* layer_flags = nullptr,
                                   int lp = 0, const int* zwrite = nullptr);

}  // namespace fvim
