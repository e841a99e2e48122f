// FP32/FP64 mixed-precision form (outer FP64 defect correction).
#include "ma_runtime.h"

using namespace mafas;

size_t mafas::mixed_bytes(const ma_params *) { return 0; }

ma_status ma_solver::mixed_allocate() { return fail(MA_ERR_ARG, "MA_MIXED is not built yet"); }

void ma_solver::mixed_release() {}

ma_status ma_solver::solve_mixed(double *, const double *, double, ma_report *)
{
    return fail(MA_ERR_ARG, "MA_MIXED is not built yet");
}
