// Solvers: RAS preconditioner (Algorithm 1), inner FP32 / outer FP64
// BiCGStab, plain FP64 BiCGStab.
#include "wcl_kernels.h"

struct Workspace {};

void wcl_free_workspace(wcl_lattice* lat) {
    delete lat->ws;
    lat->ws = nullptr;
}

extern "C" {
int wcl_block_info(const wcl_lattice*, const wcl_ras_params*, int64_t*, int64_t*) {
    wcl_set_error("not implemented");
    return WCL_ESTATE;
}
int wcl_apply_D_blocks(wcl_lattice*, const wcl_ras_params*, double, double, const void*, double*, void*) {
    wcl_set_error("not implemented");
    return WCL_ESTATE;
}
int wcl_ras_precondition(wcl_lattice*, const wcl_ras_params*, double, double, const void*, void*, int, void*) {
    wcl_set_error("not implemented");
    return WCL_ESTATE;
}
int wcl_solve_nested_bicgstab(wcl_lattice*, const wcl_solver_params*, double, double, const void*, void*, int,
                              wcl_solve_stats*, void*) {
    wcl_set_error("not implemented");
    return WCL_ESTATE;
}
int wcl_solve_bicgstab_f64(wcl_lattice*, double, int, double, double, const void*, void*, wcl_solve_stats*, void*) {
    wcl_set_error("not implemented");
    return WCL_ESTATE;
}
}
