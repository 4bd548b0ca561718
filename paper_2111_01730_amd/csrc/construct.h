// Preconditioner construction by Algorithm 1 (HODBF_invert) and Algorithm 2 (BF_SMW)
// of Section III-B, with every new butterfly reconstructed from products of existing
// operators with structured random vectors (the BF_random_matvec step).
//
// The algorithm is written once against two small interfaces: an Engine that owns
// multi-vectors (N x R, tree order, right-hand sides interleaved: element (i, q) at
// i R + q) and runs their elementwise work, and LinOps y = M x / y = M^T x (plain
// transpose).  The host engine computes in complex FP64 (the CPU-testable form); the
// device engine runs the same algorithm on the grouped-GEMM kernels.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <vector>

#include "internal.h"
#include "sketch_rng.h"

namespace hodbf {

// A multi-vector owned by an engine.
struct Mv {
  virtual ~Mv() = default;
  int R = 0;
};
using MvP = std::shared_ptr<Mv>;

// Rows [lo, hi) of the tree order, several ranges: a row set for masks.
using RowSet = std::vector<std::pair<int32_t, int32_t>>;

// One gather request: rows `rows` (tree positions) of columns [q0, q0 + k) of a
// multi-vector, written to the host as a k x rows.size() column-major block.
struct Gather {
  int32_t q0 = 0;
  std::vector<int32_t> rows;
};

class Engine;

class LinOp {
 public:
  virtual ~LinOp() = default;
  // y = M x (trans: y = M^T x); y is overwritten everywhere, x is not changed.
  virtual void apply(Engine &E, bool trans, const Mv &x, Mv &y) const = 0;
};
using OpP = std::shared_ptr<const LinOp>;

// A set of butterflies with explicit outer factors (rows o, columns s, L levels, leaves
// at level hod_level + L): y(o) += B^L W^L ... W^1 V^0 x(s) for each, zero elsewhere.
// Dense blocks: y(rows) = D x(rows) on diagonal node ranges.
struct DenseDiag {
  int32_t lo = 0;
  Mat D;  // square, column-major
};

class Engine {
 public:
  virtual ~Engine() = default;
  const Tree *tree = nullptr;
  int64_t n() const { return tree->n; }
  // widest multi-vector the engine wants to hold at once (sketch chunks)
  virtual int max_cols() const = 0;
  virtual MvP make(int R) = 0;                              // zeroed
  virtual void zero(Mv &y) = 0;
  virtual void copy(const Mv &x, Mv &y) = 0;
  virtual void axpy(cd a, const Mv &x, Mv &y) = 0;          // y += a x
  virtual void keep_rows(const RowSet &rows, Mv &y) = 0;    // zero every row outside
  // x(r, q) = random unit-modulus value (one of (+-1 +- j)/sqrt(2), from a counter-based
  // hash of (seed, r, col0 + q)) where slot_of_row[r] * k <= col0 + q < (slot + 1) * k,
  // 0 elsewhere.  slot_of_row[r] < 0: the row carries no slot.
  virtual void fill_sketch(Mv &x, const std::vector<int32_t> &slot_of_row, int64_t col0, int k,
                           uint64_t seed) = 0;
  // x(r, q) = 1 where q == col_of_row[r], 0 elsewhere (unit probes)
  virtual void fill_unit(Mv &x, const std::vector<int32_t> &col_of_row) = 0;
  // all requests into out, back to back (k values per gathered row)
  virtual void gather(const Mv &y, const std::vector<Gather> &req, int k,
                      std::vector<cd> &out) = 0;
  virtual OpP butterflies(std::vector<Butterfly> bfs) = 0;
  virtual OpP dense_diag(std::vector<DenseDiag> blocks) = 0;
};

// The random value fill_sketch writes at (row r, global column g): host and device use
// the same integer hash (sketch_rng.h), so the host can regenerate any sketch entry.
inline cd sketch_value(uint64_t seed, uint64_t r, uint64_t g) {
  double re, im;
  sketch_parts(seed, r, g, re, im);
  return cd(re, im);
}

// Drop stage rows that are never written (blocks reading only rank-0 inputs) or never
// read (outputs no later block uses), with the matching columns downstream.
void prune_butterfly(Butterfly &bf);

// ---- composite operators (backend independent) ----
OpP chain(std::vector<OpP> ops);                 // y = ops.back() ... ops[0] x
OpP lincomb(std::vector<std::pair<cd, OpP>> t);  // y = sum c_i M_i x (nullptr M_i: identity)
OpP plus_identity(OpP F);                        // y = x + F x
OpP row_mask(RowSet rows);                       // y = x on rows, 0 elsewhere

// What one reconstruction builds: for every target, a butterfly with rows at node
// (lev, oi), columns at node (lev, si) and L levels (all targets share lev and L).
struct Target {
  int64_t oi = 0, si = 0;
  int ca = 0, cb = 0;  // child indices within the parent (block tables)
  int64_t tau = 0;     // parent node index at lev - 1
};

struct RbfOpts {
  double chi = 1e-4;
  double chi_inner = 0;  // tolerance of intermediate reconstructions (0: chi)
  uint64_t seed = 1;
  int k0 = 32;        // first sketch width per slot
  int k0_side[2] = {0, 0};  // first widths of the column and row sides (0: k0)
  int oversample = 10;
  int kmax = 4096;
  // the operator is nonzero only on the target blocks (true for every use here): the
  // sketches of targets whose row (column) nodes differ share columns when no target
  // couples them
};

struct RbfStats {
  int64_t sketch_cols = 0, ids = 0, applies = 0, redone = 0;
  int max_rank = 0;
  int last_k[2] = {0, 0};  // final sketch widths of the last reconstruction (column, row side)
  // sketch products (incl. gathers), interpolative decompositions, middle fit, and
  // the engine's packing of new butterfly sets
  double seconds_apply = 0, seconds_id = 0, seconds_middle = 0, seconds_pack = 0;
};

// Reconstruct the target butterflies of M (two-sided nested form: column IDs of
// row-space sketches M^T Omega up to the middle level, row IDs of column-space sketches
// M Omega from the other side, and the middle coupling fitted by least squares) in the
// layout of Butterfly: V^0, W^1..W^L (the middle folded into the first row-side
// transfer), explicit outer factors B.
std::vector<Butterfly> reconstruct(Engine &E, const LinOp &M, int lev, int L,
                                   const std::vector<Target> &tg, const RbfOpts &o,
                                   RbfStats *st = nullptr);

// Algorithm 1 driver.  fwd_offdiag(l) returns the forward operator's butterflies of
// tree level l + 1 (the blocks Z(tau1, tau2), Z(tau2, tau1) of every level-l node) with
// explicit outer factors.  The recursion bottoms out at the nodes of leaf_level (L_H:
// the tree's leaves; higher: larger nodes), whose diagonal blocks are inverted densely
// (host FP64).  Returns, per tree level from leaf_level - 1 down to min_level, the X_tau
// butterflies (four per node, children pairs, L_H - l - 1 levels), and the dense
// inverses.
struct PrecondBuild {
  std::vector<DenseDiag> leaf_inv;
  int leaf_level = 0;
  std::vector<std::vector<Butterfly>> levels;  // levels[i] is tree level leaf_level - 1 - i
  OpP leaf_op;              // the leaf inverses as the engine's operator
  std::vector<OpP> ops;     // X of each built level as the engine's operator (same order)
  RbfStats stats;
  int64_t reconstructions = 0, woodbury = 0;
};
PrecondBuild invert_hodbf(Engine &E, const Kernel &ker, int min_level, int leaf_level,
                          const std::function<std::vector<Butterfly>(int)> &fwd_offdiag,
                          const RbfOpts &o);

// The multiplicative inverse as an operator: leaf inverses, then (I + X) for each
// level already built (levels in build order, i.e. towards the root).
OpP mult_inverse(Engine &E, OpP leaf, const std::vector<OpP> &levels);

// Host engine: complex FP64 on the CPU (small problems; tests and verification).  With
// programs = true its butterfly sets are packed into the device path's grouped-GEMM
// programs (forward and transposed) and run by a host interpreter of those descriptors.
std::unique_ptr<Engine> make_host_engine(const Tree *t, int max_cols = 512, bool programs = false);

}  // namespace hodbf
