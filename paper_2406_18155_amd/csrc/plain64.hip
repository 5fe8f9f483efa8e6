// Plain complex FP64 path (baseline): unfused, one launch per local term.
#include "internal.h"

namespace scp {

scp_status launch_plain64(scp_system* sys, const double2* psi0, double2* psiT, void* work, int S,
                          hipStream_t s) {
  (void)sys; (void)psi0; (void)psiT; (void)work; (void)S; (void)s;
  return fail(SCP_EINVAL, "FP64 plain path not available");
}

}  // namespace scp
