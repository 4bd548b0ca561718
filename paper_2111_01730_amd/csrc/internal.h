// Internal types of the hodbf library (host side).  Not part of the C ABI.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hodbf.h"

namespace hodbf {

using cd = std::complex<double>;
using cf = std::complex<float>;

// Error plumbing: internal code throws hodbf::Error; the C ABI catches it.
struct Error {
  hodbf_status code;
  std::string msg;
};
[[noreturn]] void fail(hodbf_status code, const std::string &msg);
void set_last_error(const std::string &msg);
// Progress messages on stderr when the environment sets HODBF_LOG to a non-zero value.
void logf(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

// ---------------------------------------------------------------------------
// Geometry and cluster tree T_H (Section III-A), all arrays in tree order.
struct Tree {
  int64_t n = 0;
  int depth = 0;                          // L_H
  std::vector<int32_t> perm;              // tree position -> user index
  std::vector<std::vector<int32_t>> lo;   // lo[l][i]..lo[l][i+1]: node i at level l
  std::vector<int16_t> cx, cy, cz;        // voxel coordinates per tree position
  int32_t node_lo(int l, int64_t i) const { return lo[l][i]; }
  int32_t node_hi(int l, int64_t i) const { return lo[l][i + 1]; }
};
Tree build_tree(int nx, int ny, int nz, int leaf_size);

// Entries of Z on the host in FP64 (used for sampled ID inputs).
struct Kernel {
  double kh = 0, ka = 0;
  cd k2S;                       // K(0)
  std::vector<cd> inv_eps;      // tree order
  std::vector<cd> kappa;        // tree order
  const Tree *tree = nullptr;
  cd entry(int32_t m, int32_t n) const;
};
Kernel make_kernel(const Tree &t, const std::vector<cd> &eps_user, double h, double k0);

// Interpolative decomposition by column-pivoted Householder QR (eq. (ID)).
// M: m x n column-major (overwritten).  Returns rank r; J[0..r) skeleton column
// indices; V (r x n, column-major, ld = r) with V(:, J) = I.
int id_cpqr(cd *M, int m, int n, double chi, std::vector<int> &J, std::vector<cd> &V);

// ---------------------------------------------------------------------------
// Host plan of one butterfly: factors column-major, computed in FP64 and kept in
// complex FP32 (the device copies are FP32 or narrower).
struct Mat {
  int m = 0, n = 0;
  std::vector<cf> v;  // m x n column-major
};
struct Butterfly {
  int hod_level = 0;   // level of o and s in T_H
  int64_t oi = 0, si = 0;  // row node and column node indices at hod_level
  int ca = 0, cb = 0;  // for inverse factors: child block (row child, col child)
  int64_t tau = 0;     // for inverse factors: parent node index at hod_level - 1
  int L = 0;
  std::vector<Mat> V0;                       // 2^L, r x |nu_b|
  std::vector<std::vector<Mat>> W;           // W[l] for l=1..L: 2^L blocks, index a*2^{L-l}+b
  std::vector<std::vector<int32_t>> bskel;   // 2^L skeleton column lists for B (tree pos)
  std::vector<Mat> B;                        // inverse factors only: explicit B values
};

struct FwdPlan {
  Tree tree;
  Kernel ker;
  std::vector<Butterfly> bfs;  // ordered by hod level then node
  int64_t id_count = 0;
  int max_rank = 0;
};

struct BuildOpts {
  double chi = 1e-4;
  uint64_t seed = 1;
};

// A matrix-entry source for ID construction: fills out(rows x cols) column-major.
struct EntrySource {
  virtual ~EntrySource() = default;
  virtual void fill(const int32_t *rows, int nr, const int32_t *cols, int nc, cd *out) const = 0;
  // geometric position (tree position -> voxel coords) for near-row selection
  const Tree *tree = nullptr;
};

// Compress the block (row node (lev, oi)) x (col node (lev, si)) with L levels.
// Row sampling: all rows when few, else near rows plus uniform random rows.
Butterfly build_butterfly(const EntrySource &src, const Tree &t, int lev, int64_t oi,
                          int64_t si, int L, double chi, uint64_t seed, int64_t *id_count);

FwdPlan build_forward_plan(const hodbf_build_params &p);

}  // namespace hodbf
