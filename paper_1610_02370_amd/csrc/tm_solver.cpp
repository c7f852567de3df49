// Flexible GMRES preconditioned by SAP, defect correction, and the block-shape tuner.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/tm.h"
#include "tm_api_internal.h"

using namespace tmsap;

extern "C" {

void tm_solver_opts_default(tm_solver_opts* s) {
    if (!s) return;
    std::memset(s, 0, sizeof *s);
    s->form = TM_SOLVE_FLEXIBLE;
    s->restart = 20;
    s->max_iters = 2000;
    s->n_cycles = 4;
    s->mr_iters = 4;
    for (int a = 0; a < 4; ++a) s->block_dims[a] = 4;
    s->inner_tol = 1e-6;
    s->max_outer = 50;
    s->group = 0;
}

int tm_fgmres_solve(const tm_geom*, const void*, const void*, void*, double, double, double, const tm_solver_opts*,
                    const tm_opts*, tm_solve_report*) {
    return fail(TM_ERR_ARG, "tm_fgmres_solve: not built yet");
}

int tm_autotune_sap(const tm_geom*, const void*, double, double, int, int, const tm_opts*, int*) {
    return fail(TM_ERR_ARG, "tm_autotune_sap: not built yet");
}

}  // extern "C"
