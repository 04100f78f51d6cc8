// Context object and the internal interface between the operator entry points
// and the iterative solvers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fvim.h"
#include "kernels.hpp"

namespace fvim {
struct SolverWork;
struct FricWork;
}

struct fvim_ctx {
  fvim_grid grid;
  fvim_material mat;
  int precision = 0;
  int k0_policy = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  double mu = 0, lam = 0;
  void* twx64 = nullptr;
  void* twy64 = nullptr;
  void* twx32 = nullptr;
  void* twy32 = nullptr;
  void* bufA = nullptr;
  void* bufB = nullptr;
  void* k0buf = nullptr;       // float64 plane sums and mean-mode constants (FP32 path)
  void* mt64 = nullptr;        // per-mode depth-pass constants (built on first use)
  void* mt32 = nullptr;
  double* hz = nullptr;        // non-uniform depth nodes: element lengths (device), else NULL
  double* wz = nullptr;        //   and their trapezoid weights / the uniform spacing (device)
  void* dbatch = nullptr;      // device copy of a batched depth-pass table
  size_t dbatch_bytes = 0;
  void* pbatch = nullptr;      // device copy of a persistent batched operator's table
  size_t pbatch_bytes = 0;
  // optional second stream (default priority) for the Nyquist-mode depth
  // launch beside the main one, with its fork/join events
  int use_side = 0;
  int streaming = 2;            // FVIM_OPT_STREAMING
  int persistent = 0;           // FVIM_OPT_PERSISTENT (batched applications)
  hipStream_t side = nullptr;
  hipEvent_t ev_spec = nullptr, ev_nyq = nullptr;
  size_t bufA_bytes = 0, bufB_bytes = 0, k0buf_bytes = 0;
  fvim::SolverWork* sw = nullptr;
  fvim::FricWork* fric = nullptr;   // tangential contact workspace (first use)
  // tuning: depth-pass configuration id (-1 = default for nz), and a request
  // to time every candidate on the next operator call
  int depth_cfg = -1;
  // launch choices of the four transform kernels (x_r2c, y_fwd, y_inv,
  // x_c2r) in float64 [0] and float32 [1] (default tile, radix 4 unless
  // tuned or set)
  fvim::FftChoice fft[2][4];
  std::string arch;              // gcnArchName of the device (tuning records)
  // set by the solvers of the FP32_REFINED mode for the applications that
  // must be float64 (refinement phase, right-hand sides, surface corrections)
  int force_fp64 = 0;
  // replay the contact iteration as a captured HIP graph
  int use_graphs = 1;
  int tune_pending = 0;
  // stage timing: pairs of events per launch, tagged by stage
  int timing = 0;
  struct StageEv {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<StageEv> evs;
};

namespace fvim {
// Held by every graph capture of the library (begin to end) and by every
// library call that allocates or frees device or pinned memory or copies
// synchronously.  On HIP such a call made by one thread while another
// thread captures either invalidates that capture or fails itself, so the
// library's own threads (server slots, callers solving on several streams)
// must not overlap the two.
std::recursive_mutex& device_lock();
int fail(int code, const char* msg);
int fail_hip(hipError_t e, const char* where);
int ctx_reserve(fvim_ctx* c, void** p, size_t* have, size_t need);
int operator_apply(fvim_ctx* c, const double* eps_p, const double* traction, double* strain, double* stress,
                   double* disp, double* surf_u3);
// Sizes the workspace and builds the mode tables of an application with
// eigenstrain and traction inputs and strain output, in float64 and, in the
// FP32_REFINED mode, in float32.
int operator_reserve(fvim_ctx* c, const double* eps_p, const double* traction, double* strain);
// R = x - (grad_s M[eps_p] + grad_s M[traction]) with the weighted sums of
// the residual epilogue (kernels.hpp) written as *nparts pairs to part
// (at most operator_resid_parts(c) pairs).  zact (device, may be NULL): the
// eigenstrain layers z >= *zact are zero and are skipped.
int operator_apply_resid(fvim_ctx* c, const double* eps_p, const double* traction, const double* x,
                         const double* Fo, double* R, double* part, int* nparts, const int* zact);
int operator_resid_parts(const fvim_grid& g);
// The context's transform choices of precision index prec (0 float64, 1
// float32) packed as FVIM_OPT_FFT_CONFIG encodes them; fft_pack_all packs
// both precisions (a key that changes whenever any choice does).
int fft_pack(const fvim_ctx* c, int prec);
int fft_pack_all(const fvim_ctx* c);
void solver_release(fvim_ctx* c);
size_t solver_footprint(const fvim_grid* g, size_t V);
void friction_release(fvim_ctx* c);
// Allocates the tangential contact workspace now (not inside a solve).
int friction_reserve(fvim_ctx* c);
size_t friction_footprint(const fvim_grid* g);
// warm: q_out holds a previous solution to start from (projected onto the
// new constraint set); else the start is the scaled full-slip field.
// ue: when not NULL, a tangential displacement [2][nx ny] of other loads
// added to C q (the pressure's, with the Cerruti cross terms).
int friction_solve(fvim_ctx* c, const double* p, double mu_f, double Qx, double Qy, double tol, int max_iter,
                   double* q_out, fvim_tangential_info* info, bool warm = false, const double* ue = nullptr);
// Polonsky-Keer on the context stream.  p: in warm start (all zero ->
// uniform), out solution.  gap may be NULL.
int pk_solve(fvim_ctx* c, const double* h, double W, double tol, int max_iter, double* p, double* gap,
             fvim_contact_info* info);
// Allocates the contact solver's workspace now (not inside a solve).
int solver_reserve(fvim_ctx* c);
// Normal contact with Coulomb friction into T = (q0, q1, p) [3][nx ny]:
// Goodman's sequence (coupled 0: the normal solve, then the tangential one)
// or the alternation coupled through the Cerruti cross terms (coupled 1)
// until dA sum |dp| / W + dA sum |dq| / (mu_f W) < tol.  Normal solves to
// tol_contact, tangential ones to tol_f, each at most max_contact
// iterations; at most max_iter alternations.  warm: T holds a traction to
// start from (else the pressure is still read as contact_solve's warm start
// and q is ignored).
int frictional_solve(fvim_ctx* c, const double* h, double W, double mu_f, double Qx, double Qy, int coupled,
                     double tol, double tol_contact, double tol_f, int max_contact, int max_iter, double* T,
                     bool warm, fvim_frictional_info* info);
// frictional_solve's workspaces, allocated now.
int frictional_reserve(fvim_ctx* c);
// Device bytes the Newton-Krylov solver adds when opts selects it (0 else).
size_t krylov_footprint(const fvim_grid* g, const fvim_ep_opts* o);
// out = base - T (u1 - u2) for the voxels v < na of each component
// (stride nvox; base and u2 may be NULL), T the consistent tangent of the
// radial return's d_eps_p at the strain increment d_eps.
hipError_t launch_plastic_tangent(const double* d_eps, const double* u1, const double* u2, const double* base,
                                  const double* sig_n, const double* ep_n, double* out, size_t na, size_t nvox,
                                  double lam, double mu, double sy0, double eh, hipStream_t st);
}  // namespace fvim
