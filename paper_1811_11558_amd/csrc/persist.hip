// Persistent batched operator (gfx950): the whole fused Mindlin + Boussinesq
// application over several grids of different sizes in ONE cooperative
// launch.  The grid of blocks (as many as the device holds at once) loops
// over the blocks of each stage in turn -- forward row transforms, forward
// column transforms, the depth pass with the Nyquist sign replicas, the
// Nyquist averages, inverse column and inverse row transforms -- and meets
// at a grid barrier between stages, so the stages need no launches of their
// own and no block waits for a kernel boundary.  Every block runs the same
// device bodies as the batched launches (fft_dev.hpp, depth_dev.hpp), so the
// results are bitwise those of the multi-launch batch.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "depth_dev.hpp"
#include "fft_dev.hpp"
#include "kernels.hpp"

namespace fvim {
namespace {

namespace cg = cooperative_groups;

template <typename T, int LPM, int P>
__global__ __launch_bounds__(NT) void k_op_persistent(const OpBatch* __restrict__ t) {
  __shared__ double red[NT / 64];
  cg::grid_group grid = cg::this_grid();
  const int G = (int)gridDim.x;
  const int b0 = (int)blockIdx.x;
  const XformBatch& x0 = t->x[0];
  for (int blk = b0; blk < x0.first[x0.n]; blk += G) x_r2c_batch_block<T>(x0, blk, red);
  grid.sync();
  const XformBatch& x1 = t->x[1];
  for (int blk = b0; blk < x1.first[x1.n]; blk += G) y_fwd_batch_block<T>(x1, blk);
  grid.sync();
  const DepthBatch* d = &t->d;
  for (int blk = b0; blk < d->first_main[d->n]; blk += G) depth_batch_block<T, LPM, P, false, false, false>(d, blk);
  grid.sync();
  for (int blk = b0; blk < d->first_nyq[d->n]; blk += G) nyq_batch_block<T>(d, blk);
  grid.sync();
  const XformBatch& x2 = t->x[2];
  for (int blk = b0; blk < x2.first[x2.n]; blk += G) y_inv_batch_block<T>(x2, blk);
  grid.sync();
  const XformBatch& x3 = t->x[3];
  for (int blk = b0; blk < x3.first[x3.n]; blk += G) x_c2r_batch_block<T>(x3, blk, red);
}

}  // namespace

template <typename T>
hipError_t launch_operator_persistent(OpBatch& host, OpBatch* dev, int depth_cfg, bool disp, bool wx,
                                      hipStream_t st) {
  if (disp || wx || !std::is_same<T, double>::value) return hipErrorNotSupported;
  const void* kern = nullptr;
  switch (depth_cfg) {          // the default layouts of nz <= 16, 32, 64, 128
    case 0: kern = (const void*)k_op_persistent<double, 16, 1>; break;
    case 1: kern = (const void*)k_op_persistent<double, 16, 2>; break;
    case 3: kern = (const void*)k_op_persistent<double, 32, 2>; break;
    case 5: kern = (const void*)k_op_persistent<double, 64, 2>; break;
    default: return hipErrorNotSupported;
  }
  const int cap[] = {16, 32, 0, 64, 0, 128};      // nodes per mode of those layouts
  if (host.d.n < 1 || host.d.n > DEPTH_BATCH_MAX) return hipErrorInvalidValue;
  for (int c = 0; c < host.d.n; ++c) {
    const DepthParams& q = host.d.prm[c];
    if (!q.mtab || !q.rep_out || q.hz || q.nz > cap[depth_cfg] || q.off_disp >= 0 || q.off_u3 >= 0 ||
        q.off_stress >= 0)
      return hipErrorInvalidValue;
  }
  size_t lds = 0;
  for (int k = 0; k < 4; ++k) {
    const size_t l = xform_batch_prepare<T>(k, host.x[k]);
    if (l == 0) return hipErrorInvalidValue;
    lds = std::max(lds, l);
  }
  int items = 0;
  for (int k = 0; k < 4; ++k) items = std::max(items, host.x[k].first[host.x[k].n]);
  items = std::max(items, std::max(host.d.first_main[host.d.n], host.d.first_nyq[host.d.n]));
  int device = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1 || ncu < 1) return hipErrorInvalidConfiguration;
  // every block of the grid is resident at once (the barrier needs it)
  const int grid = std::min(per_cu * ncu, std::max(items, 1));
  // pageable source: the copy is staged before the call returns
  e = hipMemcpyAsync(dev, &host, sizeof(OpBatch), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&dev};
  return hipLaunchCooperativeKernel(kern, dim3(grid), dim3(NT), args, (unsigned)lds, st);
}

template hipError_t launch_operator_persistent<double>(OpBatch&, OpBatch*, int, bool, bool, hipStream_t);
template hipError_t launch_operator_persistent<float>(OpBatch&, OpBatch*, int, bool, bool, hipStream_t);

}  // namespace fvim
