// The operator object behind the C ABI and the host-side programs that drive the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "device.h"
#include "internal.h"

namespace hodbf {

void hip_check(hipError_t e, const char *what);
#define HIPCHK(x) ::hodbf::hip_check((x), #x)

// Owning device allocation.
// A device allocation: through the allocator hook installed when it was made (release
// and ctx remembered), else hipMalloc / hipFree.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hodbf_free_fn release = nullptr;
  void *ctx = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), release(o.release), ctx(o.ctx) {
    o.p = nullptr;
    o.bytes = 0;
    o.release = nullptr;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      bytes = o.bytes;
      release = o.release;
      ctx = o.ctx;
      o.p = nullptr;
      o.bytes = 0;
      o.release = nullptr;
    }
    return *this;
  }
  ~DevBuf() { reset(); }
  void reset();
  void alloc(size_t nbytes);
  void upload(const void *src, size_t nbytes, hipStream_t st);
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
};

// One grouped-GEMM launch of a program.  X/T select the input buffers of its pairs;
// out: 0 -> T (stage workspace), 1 -> the program's output buffer.
struct Launch {
  int64_t s0 = 0, ns = 0;
  int beta = 0, out = 0;
  int64_t cls[kRowClasses + 1] = {};  // row-tile class boundaries (set at upload)
};

// A sequence of dependent grouped launches (one apply of a factor set).
struct Program {
  std::vector<Launch> launches;
  DevBuf segs, pairs, rowmap;
  int64_t t_rows = 0;  // stage workspace rows
  // vector rows one apply moves: per launch every output row once and every distinct
  // input row segment once (stacked blocks share theirs)
  int64_t io_rows = 0;
  int64_t nseg = 0, npair = 0;
};

// Host-side record of a stored block, for export and stats: element (i, k) of the
// m x n block sits at off + k * lda + i of its arena (lda > m when blocks that share
// an input are stacked).
struct BlockRec {
  int64_t kind, l, i, ca, cb, lev, a, b, m, n, off, lda;
};

struct PrecondLevel {
  Program prog;  // stages of the X_tau butterflies of one tree level + the add-into-z reduce
  int level = 0;
};

struct PrecondData {
  bool present = false;
  int min_level = 0;
  DevBuf F32, BF16, F16;     // factor arenas (complex FP32 / BF16 / FP16), same offsets
  std::vector<float> scales; // load scale of every table row
  Program leaf;              // z = D_leaf^{-1} x
  std::vector<PrecondLevel> levels;  // from level L_H - 1 towards min_level
  std::vector<BlockRec> table;
  int64_t entries = 0;
  int max_rank = 0;
  int default_ft = FT_C64;
  double seconds = 0;
  int64_t reconstructions = 0, sketch_cols = 0;  // randomized reconstructions, sketch columns
};

struct OpDevice {
  DevBuf perm;      // int32, tree position -> user index (scatter)
  DevBuf tpos;      // int32, user index -> tree position (gather)
  DevBuf xyz;       // short4 voxel coordinates, tree order
  DevBuf inv_eps;   // double2, tree order
  DevBuf kappa;     // double2, tree order
};

}  // namespace hodbf

struct hodbf_op {
  hodbf_build_params params{};
  int64_t n = 0;
  hodbf::Tree tree;
  hodbf::Kernel ker;
  hodbf::OpDevice dev;
  hodbf::DevBuf fwdF;  // complex FP32 factor arena of Z_con
  hodbf::Program fwd;
  std::vector<hodbf::BlockRec> fwd_table;
  int64_t fwd_entries = 0;
  int max_rank = 0;
  int64_t id_count = 0;
  double build_seconds = 0;
  hodbf::PrecondData pre;
};

namespace hodbf {

// Run a program on tree-order RHS-interleaved complex FP32 buffers.  For the forward
// operator X is the input, OUT the output; T is a workspace of prog.t_rows * R.
void run_program(const Program &prog, const void *F, int ftype, const float2 *X, float2 *T,
                 float2 *OUT, int R, hipStream_t st);

// y_tree = Z_con x_tree and z_tree = P x_tree on internal buffers (workspace supplied).
// ftype FT_C64 (FP32 arithmetic) or FT_C64_S3 (split-BF16 arithmetic) for the forward.
void apply_forward_tree(const hodbf_op &op, const float2 *x, float2 *y, float2 *work, int R,
                        hipStream_t st, int ftype = FT_C64);
int64_t forward_work_rows(const hodbf_op &op);
void apply_precond_tree(const hodbf_op &op, int ftype, const float2 *x, float2 *z, float2 *work,
                        int R, hipStream_t st);
int64_t precond_work_rows(const hodbf_op &op);

// One stream-ordered scratch allocation owned by a scope: it comes from the allocator
// hook installed at construction (else hipMallocAsync) and goes back to that same
// allocator when the scope ends, also when an error unwinds it.
class Scratch {
 public:
  Scratch(size_t bytes, hipStream_t st);
  ~Scratch();
  Scratch(const Scratch &) = delete;
  Scratch &operator=(const Scratch &) = delete;
  template <typename T>
  T *as() const { return static_cast<T *>(p_); }

 private:
  void *p_ = nullptr;
  hipStream_t st_;
  hodbf_free_fn release_ = nullptr;
  void *ctx_ = nullptr;
};

// Algorithm 1 / Algorithm 2 on the device; plan: the forward butterflies (host V0 / W
// values and outer-factor skeletons) the construction reads B from.
void build_precond(hodbf_op &op, const std::vector<Butterfly> &plan, hipStream_t st);

// Pack a set of butterflies (stage launches + final reduce into leaf rows) into prog.
struct PackInput {
  std::vector<const Butterfly *> bfs;
  bool forward = false;  // forward: B via device entry generation, dense leaves added
};

}  // namespace hodbf
