// Differentiable refinement on the blurred pocket density (placeholder until
// the surrogate kernels land).
#include <hip/hip_runtime.h>

#include "gd_internal.h"
#include "runtime.h"

using namespace gd;

extern "C" {

gd_status gd_surrogate_fwd(const gd_pocket*, const gd_ligands*, int32_t, const int32_t*, const float*, const float*,
                           const float*, const float*, const float*, const float*, int32_t, void*, float*) {
    clear_error();
    return fail(GD_ERR_ARG, "gd_surrogate_fwd: not available in this build");
}

gd_status gd_surrogate_bwd(const gd_pocket*, const gd_ligands*, int32_t, const int32_t*, const float*, const float*,
                           const float*, const float*, const float*, const float*, int32_t, const float*, void*,
                           float*, float*, float*) {
    clear_error();
    return fail(GD_ERR_ARG, "gd_surrogate_bwd: not available in this build");
}

gd_status gd_refine(const gd_pocket*, const gd_ligands*, int32_t, const int32_t*, float*, float*, float*,
                    const gd_refine_opts*, float, int32_t, void*, float*, int32_t*, uint8_t*, uint8_t*) {
    clear_error();
    return fail(GD_ERR_ARG, "gd_refine: not available in this build");
}

}  // extern "C"
