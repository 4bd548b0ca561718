// Preconditioner construction (placeholder until the dense-then-compress path lands).
#include "op.h"

namespace hodbf {

void build_precond(hodbf_op &op, hipStream_t st) {
  (void)op;
  (void)st;
  fail(HODBF_E_STATE, "preconditioner construction not available");
}

}  // namespace hodbf
