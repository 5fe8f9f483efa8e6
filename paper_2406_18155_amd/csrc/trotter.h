// Host launchers of the product-formula adjoint beyond those the shared
// internal header declares.
#pragma once

#include "internal.h"

namespace scp {

// The LCAM gradient (Sec. 2.5) started from psi_I(T) of the forward with the
// same order (device, complex128, S columns of D): the gate tables are built,
// the fused forward is not.  Arguments otherwise as launch_trotter_adjoint.
scp_status launch_trotter_adjoint_final(scp_system* sys, int order, int S, void* ws,
                                        const double2* psiT, const double2* cot, double* grad,
                                        hipStream_t st);

}  // namespace scp
