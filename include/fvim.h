/*
 * fvim.h -- C ABI of the MI355X (gfx950) implementation of the Fourier-
 * accelerated volume integral method for elastoplastic contact
 * (Frerot, Bonnet, Molinari, Anciaux, arXiv 1811.11558).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Geometry (Sec. 1, eqn periodic_cell; Sec. 3.1): a horizontally periodic
 * half-space cell lx x ly, depth axis z = x3 pointing INTO the body, outward
 * surface normal n = -e3.  In-plane grid x = (j lx/nx, i ly/ny); nz depth
 * nodes z_k = k lz/(nz-1) (both ends included).  nx and ny must be powers of
 * two in [4, 4096]; 2 <= nz <= 512.
 *
 * Field layout: every field pointer is a DEVICE pointer to contiguous,
 * 16-byte aligned float64 memory owned by the caller, x fastest:
 *   scalar  [nz][ny][nx]
 *   tensor  [6][nz][ny][nx]   symmetric, order (11,22,33,23,13,12), tensor
 *                             (not engineering) shear components
 *   vector  [3][nz][ny][nx]
 *   surface [ny][nx]          surface vector [3][ny][nx]
 * Tractions are forces per unit area exerted ON the body at its surface
 * (traction vector T = sigma . n of eqn traction); the contact pressure is
 * p = T . e3 >= 0.
 *
 * Execution: calls are asynchronous on the context's HIP stream unless
 * stated "blocking".  No call keeps a caller pointer after it returns.
 * Outputs must not alias inputs (return_map may write sigma_np1 over
 * sigma_n).  A context is used by one host thread at a time; different
 * contexts may run concurrently on different streams.
 *
 * Errors: every int-returning call returns FVIM_OK (0) or a negative
 * FVIM_E* code; on error the outputs are unspecified and no state passed by
 * the caller is modified, with one exception: elastoplastic_solve commits
 * each converged load step to the caller's state before it starts the next
 * (fvim_ep_info.committed says which steps were).  fvim_last_error() gives a
 * thread-local message.
 */
#ifndef FVIM_H
#define FVIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FVIM_OK = 0,
  FVIM_EINVAL = -1,   /* bad argument: sizes, NULL where required, NaN input */
  FVIM_ENOMEM = -2,   /* device allocation failed                          */
  FVIM_EHIP = -3,     /* a HIP runtime call failed                          */
  FVIM_ENOCONV = -4,  /* an iterative solve hit its iteration limit         */
  FVIM_ENODEV = -5    /* no usable gfx950 device                            */
};

/* Arithmetic of the operator kernels.  FVIM_FP64: everything in float64.
 * FVIM_FP32_REFINED: FFTs, kernel evaluation and depth recurrences in
 * float32; boundary fields, residuals, reductions, the load constraint and
 * the plastic-multiplier update stay float64. */
enum { FVIM_FP64 = 0, FVIM_FP32_REFINED = 1 };

/* Mean-traction (k = 0) part of the Boussinesq operator (Remark on the
 * fundamental mode): INCLUDE adds the laterally uniform strain of the mean
 * surface traction, EXCLUDE drops it.  The k = 0 Mindlin response is always
 * included (it is the exact laterally uniform solution). */
enum { FVIM_K0_INCLUDE = 0, FVIM_K0_EXCLUDE = 1 };

typedef struct {
  int32_t nx, ny, nz;
  double lx, ly, lz;
} fvim_grid;

/* Isotropic elasticity E, nu and linear isotropic hardening
 * f_h(e_p) = sigma_y0 + E_h e_p (Sec. 4.1). */
typedef struct {
  double E, nu, sigma_y0, E_h;
} fvim_material;

typedef struct fvim_ctx fvim_ctx;

/* Create a context: checks the grid, builds FFT twiddle tables and
 * allocates the device workspace lazily on first use.  hip_stream is a
 * hipStream_t (NULL = default stream).  Blocking. */
int fvim_create(const fvim_grid* grid, const fvim_material* mat, int precision,
                int k0_policy, void* hip_stream, fvim_ctx** out);
void fvim_destroy(fvim_ctx* ctx);
/* Replace the stream used by later calls on this context. */
int fvim_set_stream(fvim_ctx* ctx, void* hip_stream);
/* Depth nodes (Sec. 3.1 leaves their spacing free).  z: HOST array of nz
 * node depths, z[0] = 0, strictly increasing, z[nz-1] = lz (to 1e-12
 * relative), copied; NULL restores the uniform nodes z_i = i lz / (nz - 1).
 * The depth pass then integrates the P1 eigenstress exactly on these
 * elements, and the solvers' scalar products use the trapezoid weights of
 * these nodes.
 * Contexts with non-uniform nodes are rejected by
 * fvim_operator_apply_batch.  Drops the solver workspace (captured
 * evaluations bake the node table in).  Blocking.  FVIM_EINVAL for nodes
 * that break the rules above. */
int fvim_set_depth_nodes(fvim_ctx* ctx, const double* z);
/* Device bytes a context of this grid holds at most (workspace for the
 * fused operator with every output, plus solver state if asked).  Used by
 * admission control. */
size_t fvim_footprint_bytes(const fvim_grid* grid, int precision, int with_solver_state);
const char* fvim_last_error(void);
/* Library version string. */
const char* fvim_version(void);

/*
 * Mindlin operator N (eqn operators, eqn N:conv; Sec. 2.1-2.3, Sec. 3):
 * given the plastic strain eps_p (tensor field), the displacement u = N[C:eps_p]
 * of the traction-free half-space, evaluated per in-plane Fourier mode
 * (Thm 1) with the depth integrals of the P1-interpolated eigenstress done
 * exactly (eqns full_discrete_convolution, int_g0, int_g1), including the
 * local jump term (eqn jump).  Outputs (any may be NULL):
 *   strain  = sym grad u                         tensor
 *   stress  = C : (strain - eps_p)               tensor
 *   disp    = u (mean of each layer set to 0)     vector
 *   surf_u3 = u . e3 at z = 0                     surface
 * Asynchronous.
 */
int mindlin_apply(fvim_ctx* ctx, const double* eps_p, double* strain, double* stress,
                  double* disp, double* surf_u3);

/*
 * Boussinesq-Cerruti operator M (eqn operators, eqn M:conv, eqn B:fourier):
 * the field of the half-space loaded by the surface traction t ([3][ny][nx]).
 * Outputs as for mindlin_apply, with stress = C : strain.  The k = 0 mode
 * follows the context's k0 policy.  Asynchronous.
 */
int boussinesq_apply(fvim_ctx* ctx, const double* traction, double* strain, double* stress,
                     double* disp, double* surf_u3);

/*
 * Both operators in one pass: u = M[t] + N[C:eps_p] (eqn operators,
 * eqn total_strain_n).  Either input may be NULL (treated as zero).  This is
 * the operator application inside the plasticity residual.  Asynchronous.
 */
int fvim_operator_apply(fvim_ctx* ctx, const double* eps_p, const double* traction,
                        double* strain, double* stress, double* disp, double* surf_u3);

/*
 * fvim_operator_apply without any allocation, for callers that cannot
 * allocate device memory: code being captured into a HIP graph, serving
 * loops that must not call hipMalloc, harnesses that forbid it.  Same
 * arguments, kernels and results as fvim_operator_apply, but the spectrum
 * buffers and the per-mode table live in a fixed region of
 * FVIM_NOALLOC_BYTES (128 MiB) of device memory that the library reserves on
 * every device it runs on, from the first fvim_create there until the
 * process ends; the table is rebuilt there on each call.  The call makes no
 * hipMalloc, hipFree or other allocation (no depth-layout tuning, no stage
 * timing, no side stream: those options are ignored here).  Every call on
 * one device shares that region and it keeps the last call's contents:
 * calls that overlap in time on one device (different streams or threads)
 * race and give wrong results; calls ordered on one stream do not.
 * Asynchronous.  Errors: FVIM_EINVAL if the application needs more than
 * FVIM_NOALLOC_BYTES (the fused strain of a 128 x 128 x 64 float64 grid
 * needs about 110 MB), FVIM_EHIP if the region could not be set up.
 */
#define FVIM_NOALLOC_BYTES ((size_t)128 << 20)
int fvim_operator_apply_noalloc(fvim_ctx* ctx, const double* eps_p, const double* traction, double* strain,
                                double* stress, double* disp, double* surf_u3);

/*
 * Batched application (batching of grids of different sizes): the fused
 * operator of fvim_operator_apply for n contexts at once, ordered on the
 * stream of ctxs[0].  Contexts whose transform lengths nx and ny are both at
 * most 512 share one launch per in-plane transform stage (up to 8 grids per
 * launch, each with its length's default transform choice); longer ones run
 * their own transform launches with their own choices.  The depth pass of
 * up to 8 contexts runs as one launch for their regular modes and one for
 * their Nyquist modes, a table mapping each block to its grid (the layout is
 * the default one for the largest nz).  A context's results are therefore
 * the same in any batch (bitwise), and agree with its separate application
 * up to the summation order of the depth layout and transform choices
 * (bitwise when both are the defaults).  The arrays hold one device pointer
 * per context (eps_p[i] [6][nz][ny][nx], ...); an array that is NULL is not
 * requested for any context, and every requested pointer must be non-NULL.
 * All contexts must share the device and the precision.  Asynchronous.
 * Errors: FVIM_EINVAL for mismatched contexts or arguments.
 */
int fvim_operator_apply_batch(fvim_ctx* const* ctxs, int n, const double* const* eps_p,
                              const double* const* traction, double* const* strain, double* const* stress,
                              double* const* disp, double* const* surf_u3);

/*
 * J2 return mapping with linear isotropic hardening (Sec. 4.1), backward
 * Euler radial return, pointwise over V = nx*ny*nz voxels:
 *   sigma_tr = sigma_n + C : d_eps;  s = dev sigma_tr;  f = sqrt(3/2)|s| -
 *   (sigma_y0 + E_h ep_n);  if f > 0:  d_ep = f / (3 mu + E_h),
 *   d_eps_p = (3 d_ep / (2 sqrt(3/2)|s|)) s,  else 0;
 *   sigma_np1 = sigma_tr - 2 mu d_eps_p.
 * d_eps, sigma_n, d_eps_p, sigma_np1: tensor fields; ep_n, d_ep: scalar
 * fields.  sigma_np1 may be NULL or equal to sigma_n.  Asynchronous.
 */
int return_map(fvim_ctx* ctx, const double* d_eps, const double* sigma_n, const double* ep_n,
               double* d_eps_p, double* d_ep, double* sigma_np1);

typedef struct {
  int iters;
  double rel_change;      /* last dA * sum |p_k - p_(k-1)| / W                 */
  double kkt_residual;    /* max(|gap| on the contact set, -min gap) / max|h|, */
                          /* gap = u3 - h minus its mean on the contact set    */
  double contact_fraction;
  double mean_gap;        /* rigid approach (mean of u3 - h on the contact set) */
} fvim_contact_info;

/*
 * Frictionless normal contact of the elastic half-space with the rigid
 * surface h ([ny][nx], measured along +e3) under total load W (eqn
 * total_pressure), as the Kalker dual minimisation solved by the
 * Polonsky-Keer projected conjugate gradient (Sec. 5.1).  The compliance is
 * u3 = M[p] . e3 at z = 0: 2 / (E* |q|) per mode, mode 0 dropped.
 * p ([ny][nx]) is read as a warm start (all zero -> uniform W / area) and
 * overwritten with the solution; gap (may be NULL) receives u3 - h - mean
 * gap.  Stops when dA * sum |dp| / W < tol or max_iter is reached
 * (FVIM_ENOCONV; p then holds the last iterate).  Blocking; info on host.
 */
int contact_solve(fvim_ctx* ctx, const double* h, double W, double tol, int max_iter,
                  double* p, double* gap, fvim_contact_info* info);

typedef struct {
  int iters;
  double rel_change;      /* last dA * sum |q_k - q_(k-1)| / (mu_f W)           */
  double stick_fraction;  /* of the contact points (p > 0)                       */
  double shift[2];        /* rigid tangential shift: u_t on the stick zone       */
} fvim_tangential_info;

/*
 * Tangential contact with Coulomb friction under the normal pressure p
 * ([ny][nx], device, >= 0 (negative values count as 0), e.g. from
 * contact_solve): the friction Sec. 5.1 says
 * the contact step can include, here with normal and tangential problems
 * uncoupled (Goodman's approximation).  The tangential surface traction q
 * ([2][ny][nx], device, output; the tangential part of the traction input
 * of boussinesq_apply) minimises the complementary energy 1/2 <q, C q> over
 * |q| <= mu_f p pointwise with dA * sum q = (Qx, Qy), C the tangential block
 * of the surface compliance: (2 (1 + nu) / (E |k|)) (I - nu n n^T) per mode,
 * mode 0 dropped.  Optimality is partial slip: one rigid shift (info.shift)
 * of the stick zone, slip against q on the friction limit.  Accelerated
 * projected gradient with restart; stops when info.rel_change < tol
 * (checked every 8 iterations) or after max_iter (FVIM_ENOCONV, q holds
 * the last iterate).  Needs |Q| < mu_f W, W = dA * sum p (FVIM_EINVAL
 * otherwise; full sliding is q = mu_f p Q / |Q|).  Blocking; info (may be
 * NULL) on host.
 */
int tangential_solve(fvim_ctx* ctx, const double* p, double mu_f, double Qx, double Qy, double tol,
                     int max_iter, double* q, fvim_tangential_info* info);

typedef struct {
  int iters;              /* alternations of the normal and tangential solves */
                          /* (1 with coupled = 0)                             */
  int contact_iters;      /* Polonsky-Keer iterations over all alternations   */
  int tangential_iters;   /* tangential iterations over all alternations      */
  double rel_change;      /* last dA sum |dp| / W + dA sum |dq| / (mu_f W)    */
                          /* between alternations (coupled = 1; else inf)     */
  double kkt_residual;    /* of the last normal solve, on the surface it saw  */
                          /* (h - u3 of the tangential traction)              */
  double stick_fraction;  /* of the last tangential solve                     */
  double shift[2];        /* rigid tangential shift of the stick zone         */
} fvim_frictional_info;

/*
 * Normal contact under total load W with Coulomb friction and total
 * tangential force (Qx, Qy), |Q| < mu_f W: the friction Sec. 5.1 says the
 * contact step can include, with the normal and tangential problems coupled
 * through the Boussinesq-Cerruti surface response (eqn B:fourier: the
 * off-diagonal normal/tangential terms of B_00 and B_10, nonzero for
 * nu < 1/2).  Per in-plane mode the tangential surface displacement of a
 * pressure is u_a = K_a p and the normal displacement of a tangential
 * traction u3 = sum_a conj(K_a) q_a, K_a = i (1 - 2 nu) k_a / (2 mu |k|^2)
 * (zero at k = 0 and on the Nyquist line of axis a).
 * coupled = 1: the pressure solves contact_solve's problem on h - u3[q],
 * q solves tangential_solve's problem with the extra displacement u_t[p];
 * the two solves alternate (each warm-started from the last) until
 * dA sum |dp| / W + dA sum |dq| / (mu_f W) < tol (the normal solves run to
 * max(tol / 10, 1e-15), the tangential ones to tol), at most max_iter
 * alternations (FVIM_ENOCONV; traction then holds the last one).
 * coupled = 0: Goodman's approximation, contact_solve then tangential_solve
 * under its pressure (max_iter unused).
 * h: [ny][nx] device, as for contact_solve.  traction: [3][ny][nx] device,
 * (q1, q2, p), overwritten with the solution; warm != 0: it holds a
 * traction to start from (e.g. the solution under a nearby load), else only
 * its pressure plane is read, as contact_solve's warm start.  FVIM_EINVAL
 * for mu_f <= 0, W <= 0, |Q| >= mu_f W or bad tolerances.  Blocking; info
 * (may be NULL) on host.
 */
int frictional_contact_solve(fvim_ctx* ctx, const double* h, double W, double mu_f, double Qx, double Qy,
                             int coupled, double tol, int max_iter, int warm, double* traction,
                             fvim_frictional_info* info);

typedef struct {
  int iters;               /* contact solves (cohesive-set updates)            */
  int contact_iters;       /* Polonsky-Keer iterations over all solves         */
  double cohesive_fraction;/* of the surface points: gap <= h0                 */
  double contact_fraction; /* of the surface points: repulsive pressure > 0    */
  double adhesive_force;   /* sigma0 dA |C|                                    */
  double kkt_residual;     /* of the last contact solve                        */
} fvim_adhesive_info;

/*
 * Adhesive normal contact under total load W: the adhesion Sec. 5.1 says
 * the contact step can include, as a Dugdale cohesive zone.  The surfaces
 * attract with the stress sigma0 wherever the gap is at most the range h0
 * (the contact zone included; work of adhesion sigma0 h0); where they touch,
 * a repulsive pressure p_c >= 0 acts (Hertz-Signorini-Moreau conditions on
 * p_c).  The traction on the body is p = p_c - sigma0 1[gap <= h0] and
 * dA sum p = W.  Solved by fixed point on the cohesive set C from C = {}:
 * contact_solve's problem on h + sigma0 M[1_C] under W + sigma0 dA |C| (to
 * tol, warm-started from the previous solve), then C = {gap <= h0}, until
 * the set repeats (at most max_iter solves; FVIM_ENOCONV otherwise, p then
 * holding the last solve's traction).  sigma0 = 0 is frictionless contact.
 * h, p (output), gap (output, may be NULL): [ny][nx] device.  FVIM_EINVAL
 * for negative sigma0 or h0, and when W + sigma0 dA |C| is not positive.
 * Blocking; info (may be NULL) on host.
 */
int adhesive_contact_solve(fvim_ctx* ctx, const double* h, double W, double sigma0, double h0, double tol,
                           int max_iter, double* p, double* gap, fvim_adhesive_info* info);

/* Elastoplastic state S_n kept between load steps (Sec. 4.2, Alg. 1):
 * device pointers, caller-owned.  eps_p, sigma: tensor fields; ep: scalar
 * field; traction: surface vector [3][ny][nx]; u3p: surface residual
 * displacement [ny][nx] accumulated over the steps. */
typedef struct {
  double* eps_p;
  double* ep;
  double* sigma;
  double* traction;
  double* u3p;
} fvim_state;

typedef struct {
  double tol_outer;    /* Alg. 1 epsilon_tol on |dU3p - dU3p_prev| / |H0|   */
  double relax;        /* Alg. 1 lambda in ]0, 1]                            */
  double tol_plastic;  /* DF-SANE: |R| <= tol * max(|R0|, |grad_s M[dT]|)   */
  double tol_contact;  /* contact_solve tol                                  */
  int max_outer, max_plastic, max_contact;
  int solver;          /* 0 = DF-SANE (Sec. 4.3), 1 = Picard fixed point,    */
                       /* 2 = Newton-Krylov with the consistent tangent of */
                       /* the radial return (the alternative Sec. 4.3      */
                       /* names): GMRES without restart for each step,     */
                       /* Eisenstat-Walker forcing terms, backtracking on  */
                       /* |R|; residuals in float64, Jacobian products in  */
                       /* the operator precision; its basis adds           */
                       /* (krylov_dim + 2) * 6 nvox doubles                */
  int literal_alg1;    /* 1: overwrite the relaxed update as printed; 0:   */
                       /* keep it (plain under-relaxation, same fixed pt) */
  int anderson_m;      /* 0: Alg. 1 relaxation; 1..6: Anderson acceleration */
                       /* of the same outer fixed point with that history  */
                       /* depth and damping relax (Walker & Ni 2011); the  */
                       /* stopping test is unchanged; ignored if literal   */
  int warm_start;      /* 1: outer passes after a step's first start the    */
                       /* plasticity iteration from the previous pass's     */
                       /* solution plus the change of M[dT] (its plastic    */
                       /* part kept); 0: from the elastic trial M[dT]       */
  double inner_rel;    /* > 0: inexact plasticity solves to the relative    */
                       /* tolerance max(tol_plastic, inner_rel * the        */
                       /* previous pass's outer error) while that error is  */
                       /* at least tol_outer (with friction, the tangential */
                       /* solves likewise); a step is accepted only after a */
                       /* pass solved to the full tolerances; 0: always     */
                       /* tol_plastic                                      */
  int krylov_dim;      /* Newton-Krylov: Arnoldi steps per Newton step,     */
                       /* 1..30 (0 = 20); ignored by the other solvers      */
  double mu_f;         /* > 0: Coulomb friction in the contact step: after  */
                       /* each normal solve, tangential_solve for the total */
                       /* tangential force q_ratio * mu_f * W (|q_ratio|<1) */
                       /* to the tolerance max(tol_contact, 1e-13) (its    */
                       /* iterations count in contact_iters), and the     */
                       /* traction T carries it (none at a zero load); 0: */
                       /* frictionless                                      */
  double q_ratio[2];
  int coupling;        /* 0: Algorithm 1 (relaxation, or Anderson with      */
                       /* anderson_m); 1: its fixed point G(x) = x on the   */
                       /* surface correction x by Newton-Krylov: GMRES on   */
                       /* (J_G - I) d = x - G(x) to the Eisenstat-Walker    */
                       /* forcing term (in [1e-3, 0.5]), J_G v formed by   */
                       /* forward differences of G (one full pass each,     */
                       /* started from the pass at x), steps halved until   */
                       /* |G(x) - x| decreases; same stopping test and      */
                       /* fixed point; inner solves always to tol_plastic   */
                       /* and tol_contact; max_outer bounds Newton steps;   */
                       /* 2: Algorithm 1 until the passes it still needs,   */
                       /* extrapolated from its error's rate over the last  */
                       /* 10 passes (from pass 20 on), exceed 100; then the */
                       /* Newton coupling from its next iterate (warm from  */
                       /* its last pass); outer_iters counts both;          */
                       /* 1 and 2 add 12 nx ny nz + (coupling_krylov + 10)  */
                       /* nx ny doubles                                     */
  int coupling_krylov; /* GMRES steps per Newton step, 1..30 (0 = 10)       */
  int cerruti;         /* 1 (with mu_f > 0): the contact step couples the   */
                       /* normal and tangential problems through the        */
                       /* Boussinesq-Cerruti cross terms, as                */
                       /* frictional_contact_solve with coupled = 1 and its */
                       /* tolerance the tangential one above (alternations  */
                       /* warm-started from the previous pass's traction,   */
                       /* at most 200); 0: Goodman's uncoupled sequence     */
  double adh_sigma0;   /* > 0: adhesion in the contact step: the Dugdale    */
  double adh_h0;       /* cohesive zone of adhesive_contact_solve (stress   */
                       /* adh_sigma0, range adh_h0; cohesive set from {} at */
                       /* each pass, contact solves to tol_contact, at most */
                       /* 200 set updates); T3 is its total traction.  Not  */
                       /* with friction (FVIM_EINVAL); 0: no adhesion       */
} fvim_ep_opts;

typedef struct {
  int outer_iters;     /* Algorithm 1 passes, or Newton steps (coupling 1)  */
  int plastic_iters, contact_iters, r_evals;
  double outer_err, plastic_res;
  double kkt;          /* KKT certificate of the step's last contact solve   */
                       /* (fvim_contact_info.kkt_residual, on the surface   */
                       /* that solve saw: h - U3p_n - the relaxed correction) */
  int committed;       /* 1: the step converged and its state update was     */
                       /* applied to the caller's state; 0: not (the step   */
                       /* that failed, and every later one, is not run)     */
} fvim_ep_info;

/*
 * Algorithm 1 (alternating contact / plasticity coupling, Sec. 5.2) over
 * n_steps cumulative loads W_steps (host array).  Per step: contact on the
 * modified surface h - U3p (Remark rem:modified_contact), the incremental
 * plasticity fixed point R[d_eps] = 0 (eqn incremental_strain) solved by
 * DF-SANE or Picard, the surface residual displacement of N[C:d_eps_p],
 * relaxation, until the outer error is below tol_outer; then the state is
 * updated in place.  info: host array of n_steps records (all cleared on
 * entry).  Each converged step is committed to the state before the next
 * starts: on an error (e.g. FVIM_ENOCONV at step k) the state holds the
 * result of steps 0 .. k-1, and info[j].committed is 1 exactly for those.
 * Blocking.
 */
int elastoplastic_solve(fvim_ctx* ctx, const double* h, const double* W_steps, int n_steps,
                        const fvim_ep_opts* opts, fvim_state* state, fvim_ep_info* info);

/*
 * Stage timing (profiling aid).  With timing on, every operator application
 * records a HIP event before and after each kernel launch on the context
 * stream.  fvim_stage_times synchronises the stream, adds the elapsed time of
 * each stage over all applications since the last call into ms[stage] and
 * the number of launches into count[stage] (arrays of FVIM_NSTAGES, host
 * memory, caller-owned), then clears the record.  Stages:
 */
enum {
  FVIM_STAGE_XFWD = 0,   /* x transform of the eigenstrain and traction planes */
  FVIM_STAGE_YFWD = 1,   /* y transform of the same planes               */
  FVIM_STAGE_XFWD_T = 2, /* unused (the traction planes are part of XFWD) */
  FVIM_STAGE_YFWD_T = 3, /* unused (part of YFWD)                        */
  FVIM_STAGE_DEPTH = 4,  /* per-mode depth pass (with the sign replicas   */
                         /* of the Nyquist modes unless the side stream  */
                         /* is on)                                       */
  FVIM_STAGE_YINV = 5,   /* inverse y transform of the output planes     */
  FVIM_STAGE_XINV = 6,   /* inverse x transform of the output planes     */
  FVIM_STAGE_DEPTH_NYQ = 7, /* Nyquist modes: average of their sign      */
                            /* replicas (side stream: their depth pass)  */
  FVIM_NSTAGES = 8
};
int fvim_set_timing(fvim_ctx* ctx, int on);

/*
 * Tuning options.  FVIM_OPT_DEPTH_CONFIG: id of the depth-pass thread layout
 * (lanes per mode x nodes per lane; -1 = built-in default for nz); ids that
 * do not serve nz are rejected with FVIM_EINVAL.  FVIM_OPT_TUNE = 1: the next
 * operator call times every valid layout on its own data (blocking) and
 * keeps the fastest.  Different layouts change only the summation order.
 * Callers that need run-to-run identical results store the chosen id and
 * set it explicitly.  FVIM_OPT_GRAPHS (default 1): the contact iteration is
 * captured once as a HIP graph and replayed (same kernels, same results; 0
 * launches the kernels one by one).  FVIM_OPT_SIDE_STREAM (default 0): 1 runs
 * the Nyquist-mode depth launch on a second library stream beside the main
 * depth launch (same results).  FVIM_OPT_STREAMING (default 2): each operator
 * launch reads its input spectrum for the last time; 1 does so with streaming
 * (non-temporal) loads, which keep the previous launch's output in the
 * caches for the next one; 0 never; 2 when the spectrum buffer of the
 * application is larger than 64 MiB and at most 256 MiB (it then fits the
 * last-level cache), where that measured faster on MI355X (same results
 * either way).  FVIM_OPT_FFT_CONFIG: launch choices of the four in-plane
 * transform kernels for the context's operator precision, 3 bits each
 * (bits 3k .. 3k+2 for k = 0 forward row, 1 forward column, 2 inverse
 * column, 3 inverse row transform): tile (0: half the default LDS tile,
 * 1: default, 2: twice) | 4 for radix-8 stages (else radix 4); 0x249 is
 * the default.  Alternatives exist for transform lengths 32 .. 1024; other
 * lengths run the default.  FVIM_OPT_TUNE also times these (6 choices per
 * kernel, on the next operator call's own data) and keeps the fastest; the
 * result is recorded for the process under (nx, ny, nz, input and output
 * planes, precision, device architecture) and reused by later contexts
 * that ask for tuning.  Choices change only the summation order of the
 * transforms.  FVIM_OPT_PERSISTENT (default 0; read from the first context
 * of fvim_operator_apply_batch): 1 runs a qualifying batch (float64, strain
 * output only, every transform length <= 512, at most 8 grids, nz <= 128)
 * as ONE cooperative persistent launch whose blocks loop over every stage
 * with a grid barrier between stages; results are bitwise those of the
 * multi-launch batch, and other batches take the multi-launch path.
 */
enum { FVIM_OPT_DEPTH_CONFIG = 1, FVIM_OPT_TUNE = 2, FVIM_OPT_GRAPHS = 3, FVIM_OPT_SIDE_STREAM = 4,
       FVIM_OPT_STREAMING = 5, FVIM_OPT_FFT_CONFIG = 6, FVIM_OPT_PERSISTENT = 7 };
int fvim_set_option(fvim_ctx* ctx, int key, int value);
int fvim_get_option(fvim_ctx* ctx, int key, int* value);
int fvim_stage_times(fvim_ctx* ctx, double* ms, int* count);

/*
 * Continuous-batching solve server.
 *
 * A request is one elastoplastic contact solve (Algorithm 1 over n_steps
 * cumulative loads) on its own grid; its inputs are copied at submission.
 * Admission: a request starts when one of max_slots worker slots is free and
 * its device footprint (fvim_request_bytes) fits in what remains of
 * hbm_budget_bytes; the first pending request in submission order that fits
 * is taken.  Each slot runs on its own HIP stream (default priority), so
 * admitted requests overlap on the device while others keep arriving.  State
 * stays in device memory from admission to completion.  A slot keeps the
 * context and state memory of its last request and reuses them for a later
 * request with the same grid, material, precision and depth nodes (nothing
 * is allocated then); kept memory counts against the budget and is given
 * back when a pending request does not fit otherwise.  A request's result
 * does not depend on the other requests in flight nor on the slot's previous
 * request (same kernels, default depth-pass layout, deterministic
 * reductions, state cleared).
 * Times are seconds since the server was created.  Results stay owned by the
 * server until fvim_server_release.  Thread-safe.
 */
#define FVIM_MAX_STEPS 16
typedef struct {
  fvim_grid grid;
  fvim_material mat;
  int precision;
  int n_steps;
  double W_steps[FVIM_MAX_STEPS];
  fvim_ep_opts opts;
  const double* h;           /* HOST pointer [ny][nx], copied at submission */
  const double* z;           /* HOST [nz] depth nodes (fvim_set_depth_nodes  */
                             /* rules) or NULL (uniform), copied            */
} fvim_request;

typedef struct {
  int status;                /* FVIM_OK or the solve's error code           */
  double t_submit, t_admit, t_done;
  fvim_ep_info info;         /* of the last load step; of the failing step   */
                             /* when status is not FVIM_OK                  */
  double contact_fraction;   /* of the final pressure                       */
  const double* p;           /* HOST [ny][nx] final contact pressure        */
  const double* u3p;         /* HOST [ny][nx] final surface residual disp.  */
  char error[160];           /* message of a failed solve ("" when status 0) */
} fvim_result;

typedef struct {
  int pending, running;
  uint64_t completed;
  size_t bytes_in_use;       /* footprints of running requests and of the   */
                             /* contexts idle slots keep                    */
  size_t peak_bytes, budget;
} fvim_server_stats;

typedef struct fvim_server fvim_server;

/* Index of the request the admission rule takes from pending footprints
 * (first that fits in budget - in_use), or -1.  Pure function. */
int fvim_admit_index(const size_t* pending_bytes, int n, size_t budget, size_t in_use);
/* Device bytes a request holds while it runs (0 for an invalid grid). */
size_t fvim_request_bytes(const fvim_request* r);
int fvim_server_create(size_t hbm_budget_bytes, int max_slots, int device, fvim_server** out);
/* FVIM_ENOMEM if the request can never fit the budget. */
int fvim_server_submit(fvim_server* s, const fvim_request* r, uint64_t* id);
/* Returns 1 and fills out when done, 0 while pending or running (wait = 1
 * blocks until done), or a negative error code for an unknown id. */
int fvim_server_poll(fvim_server* s, uint64_t id, int wait, fvim_result* out);
int fvim_server_release(fvim_server* s, uint64_t id);
int fvim_server_get_stats(fvim_server* s, fvim_server_stats* out);
/* Finishes every submitted request, then frees the server. */
void fvim_server_destroy(fvim_server* s);

#ifdef __cplusplus
}
#endif
#endif /* FVIM_H */
