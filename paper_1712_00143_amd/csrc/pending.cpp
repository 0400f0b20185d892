// Entry points whose kernels are not built yet: they fail cleanly.
#include "solver.h"

extern "C" {

#define PENDING(name, ...)                                                   \
    hisq_status name(__VA_ARGS__) { return set_err(nullptr, HISQ_ERR_STATE, #name " is not built yet"); }

PENDING(hisq_ptc_create, hisq_lattice, int, const int *, hisq_ptc *)
PENDING(hisq_ptc_destroy, hisq_ptc)
PENDING(hisq_ptc_set_weights, hisq_ptc, const double *)
PENDING(hisq_ptc_get_weights, hisq_ptc, double *)
PENDING(hisq_ptc_layer_forward, hisq_ptc, int, const void *, void *, int)
PENDING(hisq_ptc_layer_backward, hisq_ptc, int, const void *, const void *, void *, double *, int)
PENDING(hisq_ptc_apply, hisq_ptc, const void *, void *, int)
PENDING(hisq_ptc_harvest, hisq_ptc, hisq_lattice, double, const double *, int, int, int *)
PENDING(hisq_ptc_train, hisq_ptc, int, int, double, unsigned long long, double *)
PENDING(hisq_cg_learned, hisq_lattice, hisq_ptc, double, const double *, double *,
        const hisq_solver_params *, hisq_solver_info *)
}
