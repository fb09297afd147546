// Reverse-mode derivative of the radiative-transfer subcycle.
#include <hip/hip_runtime.h>

#include "rt.h"
#include "rt_internal.hpp"

extern "C" int rt_subcycle_adjoint(const rt_state* initial, int n_subcycles, int checkpoint_every,
                                   const double* dL_dxHI_final, double* dL_dlnQ, double* dL_dln_nH,
                                   void* hip_stream) {
    (void)initial; (void)n_subcycles; (void)checkpoint_every; (void)dL_dxHI_final; (void)dL_dlnQ;
    (void)dL_dln_nH; (void)hip_stream;
    return rt_fail(RT_ESTATE, "rt_subcycle_adjoint is not available in this build");
}
