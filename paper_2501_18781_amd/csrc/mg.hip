// mg.hip -- FP32 geometric multigrid pieces (placeholder until implemented).
#include "mf.h"
#include "kernels.hpp"

extern "C" {
mf_status mf_mg_create(mf_ctx *, const mf_operator *, const mf_mg_params *, mf_mg **mg, mf_stream)
{
    if (mg) *mg = nullptr;
    return MF_ERR_STATE;
}
void mf_mg_destroy(mf_mg *) {}
int32_t mf_mg_n_levels(const mf_mg *) { return 0; }
mf_status mf_mg_lambda_max(const mf_mg *, double *) { return MF_ERR_STATE; }
mf_status mf_mg_vcycle(mf_mg *, const double *, double *, mf_stream) { return MF_ERR_STATE; }
mf_status mf_mg_cg_solve(mf_mg *, const double *, double *, double, int32_t, mf_solve_info *, mf_stream)
{
    return MF_ERR_STATE;
}
}
