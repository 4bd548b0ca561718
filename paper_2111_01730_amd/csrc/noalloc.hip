// hodbf_apply_noalloc: y = Z_con x like hodbf_apply, with every temporary (the
// tree-order copies of x and y and the stage workspace) in one file-scope device array
// instead of allocations, for callers that cannot allocate.  Each GPU holds its own
// copy of the array for the life of the process; its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "op.h"
#include "precond_host.h"

namespace hodbf {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;

// the scratch array; host code uses the per-device address below, never this name
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device id, null until looked up

void *scratch_on_current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev >= int(g_scratch_ptr.size())) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[size_t(dev)]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(HODBF_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[size_t(dev)] = p;
  }
  return g_scratch_ptr[size_t(dev)];
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

}  // namespace hodbf

using namespace hodbf;

extern "C" hodbf_status hodbf_apply_noalloc(const hodbf_op *op, int32_t nrhs, hodbf_dtype dtype,
                                            const void *x, int64_t ldx, void *y, int64_t ldy,
                                            void *stream) {
  return hodbf_guarded([&] {
    if (!op) fail(HODBF_E_ARG, "NULL operator");
    if (nrhs < 0) fail(HODBF_E_ARG, "nrhs < 0");
    if (dtype != HODBF_C64 && dtype != HODBF_C128) fail(HODBF_E_ARG, "unknown dtype");
    if (nrhs == 0) return;
    if (!x || !y) fail(HODBF_E_ARG, "NULL vector");
    if (ldx < op->n || ldy < op->n) fail(HODBF_E_ARG, "leading dimension < N");
    const size_t es = dtype == HODBF_C128 ? 16 : 8;
    const char *xb = static_cast<const char *>(x), *yb = static_cast<const char *>(y);
    const char *xe = xb + es * size_t(ldx * (nrhs - 1) + op->n);
    const char *ye = yb + es * size_t(ldy * (nrhs - 1) + op->n);
    if (xb < ye && yb < xe) fail(HODBF_E_ARG, "x and y overlap");
    const size_t vbytes = round256(size_t(op->n) * size_t(nrhs) * sizeof(float2));
    const size_t wbytes =
        round256(size_t(std::max<int64_t>(forward_work_rows(*op), 1)) * size_t(nrhs) * sizeof(float2));
    const size_t need = 2 * vbytes + wbytes;
    if (need > kScratchBytes)
      fail(HODBF_E_ARG, "hodbf_apply_noalloc needs " + std::to_string(need) +
                            " bytes of scratch for these sizes; the static scratch holds " +
                            std::to_string(kScratchBytes) + " (use fewer right-hand sides)");
    char *base = static_cast<char *>(scratch_on_current_device());
    hipStream_t st = static_cast<hipStream_t>(stream);
    float2 *xt = reinterpret_cast<float2 *>(base);
    float2 *yt = reinterpret_cast<float2 *>(base + vbytes);
    float2 *wk = reinterpret_cast<float2 *>(base + 2 * vbytes);
    const bool c128 = dtype == HODBF_C128;
    // every element of xt, the workspace rows each stage reads and yt are written before
    // they are read (gather, then the program's launches, the last one covering every
    // row of y through the dense leaf blocks), so nothing needs clearing
    launch_gather(x, c128, ldx, xt, false, op->dev.tpos.as<int32_t>(), op->n, nrhs, st);
    apply_forward_tree(*op, xt, yt, wk, nrhs, st);
    launch_scatter(yt, false, y, c128, ldy, op->dev.perm.as<int32_t>(), op->n, nrhs, st);
    HIPCHK(hipGetLastError());
  });
}
