"""MI355X (gfx950) implementation of the Fourier-accelerated volume integral
method for elastoplastic contact (Frerot, Bonnet, Molinari, Anciaux,
arXiv 1811.11558).

The compute path is the HIP library ``libfvim.so`` (sources in ``csrc/``,
ABI in ``include/fvim.h``); this package is a thin ctypes binding that
passes torch device pointers and the current HIP stream.  Importing the
package does not load the library; the first call does, and raises if it has
not been built (``python -m paper_1811_11558_amd.build``).
"""
from .binding import (Context, FvimError, load_library, contact_info_dict,
                      EPOptions, mindlin_apply, boussinesq_apply, operator_apply,
                      return_map, contact_solve, tangential_solve, frictional_contact_solve, adhesive_contact_solve,
                      elastoplastic_solve, Server,
                      admit_index, request_bytes, operator_apply_batch,
                      operator_apply_noalloc, NOALLOC_BYTES)

__all__ = ["Context", "FvimError", "load_library", "contact_info_dict", "EPOptions",
           "mindlin_apply", "boussinesq_apply", "operator_apply", "return_map",
           "contact_solve", "tangential_solve", "frictional_contact_solve", "adhesive_contact_solve", "elastoplastic_solve", "Server", "admit_index", "request_bytes",
           "operator_apply_batch", "operator_apply_noalloc", "NOALLOC_BYTES"]
