// Host-side pieces of the preconditioner construction shared by the device build and
// the host-only probe, and the exception guard every C entry point runs under.
#pragma once

#include <new>
#include <stdexcept>
#include <vector>

#include "construct.h"
#include "op.h"

namespace hodbf {

// Butterflies of tree level l + 1 of the forward plan (the blocks Z(tau1, tau2) and
// Z(tau2, tau1) of every level-l node), outer factors B^L filled from the kernel
// entries; ca / cb / tau set to the children and their parent.
std::vector<Butterfly> forward_offdiag_explicit(const Tree &t, const std::vector<Butterfly> &plan,
                                               const Kernel &ker, int l);

// Block table (rows of BlockRec) and values of a host-built preconditioner: leaf
// inverses as kind 0 at the recursion's leaf level, every X_tau butterfly's V^0 / W / B blocks with
// (l, i, ca, cb) = (tree level of tau, tau, child row, child column).
void export_precond_build(const PrecondBuild &pb, std::vector<BlockRec> &table,
                          std::vector<cd> &vals);

}  // namespace hodbf

// Runs f, turning internal errors into a status and the thread's last-error message.
template <typename F>
hodbf_status hodbf_guarded(F &&f) {
  try {
    f();
    return HODBF_OK;
  } catch (const hodbf::Error &e) {
    hodbf::set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    hodbf::set_last_error("host allocation failed");
    return HODBF_E_NOMEM;
  } catch (const std::exception &e) {
    hodbf::set_last_error(e.what());
    return HODBF_E_HIP;
  } catch (...) {
    hodbf::set_last_error("unknown internal error");
    return HODBF_E_HIP;
  }
}
