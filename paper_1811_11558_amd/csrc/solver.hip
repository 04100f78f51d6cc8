// Iterative solvers on top of the operators: Polonsky-Keer contact and the
// Algorithm 1 coupling with the DF-SANE plasticity fixed point.
#include "common.hpp"
#include "kernels.hpp"
#include "solver.hpp"

namespace fvim {

struct SolverWork {
  int dummy;
};

void solver_release(fvim_ctx* c) {
  delete c->sw;
  c->sw = nullptr;
}

size_t solver_footprint(const fvim_grid* g, size_t V) { return 0; }

}  // namespace fvim

extern "C" {

int contact_solve(fvim_ctx* c, const double* h, double W, double tol, int max_iter, double* p, double* gap,
                  fvim_contact_info* info) {
  return fvim::fail(FVIM_EINVAL, "contact_solve: not available in this build");
}

int elastoplastic_solve(fvim_ctx* c, const double* h, const double* W_steps, int n_steps, const fvim_ep_opts* opts,
                        fvim_state* state, fvim_ep_info* info) {
  return fvim::fail(FVIM_EINVAL, "elastoplastic_solve: not available in this build");
}

}  // extern "C"
