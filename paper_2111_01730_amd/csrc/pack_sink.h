// Accumulator used while packing butterfly factors into a device program.
#pragma once

#include <functional>
#include <vector>

#include "op.h"

namespace hodbf {

struct PackSink {
  std::vector<Seg> segs;
  std::vector<Pair> pairs;
  std::vector<RowMap> rowmap;
  std::vector<Launch> launches;
  int64_t t_rows = 0;
  std::vector<BlockRec> *table = nullptr;
  // host-valued block -> arena offset; sets the block's load scale
  std::function<int64_t(const Mat &, float *)> put_host;
  std::vector<float> *scales = nullptr;                   // per table row, if wanted
  std::function<int64_t(int64_t, int64_t)> reserve_dev;  // device-generated block -> offset
  std::vector<EntryJob> *jobs = nullptr;
  std::vector<int32_t> *jobcols = nullptr;
};

void pack_group(PackSink &pk, const Tree &t, const std::vector<const Butterfly *> &bfs,
                bool forward, int final_beta,
                const std::function<void(const Butterfly &, int64_t *)> &meta);
// y = M^T x for a set of butterflies of one shape (the stages reversed, factors
// transposed; the last launch writes y's column-leaf rows with beta 0).
void pack_group_t(PackSink &pk, const Tree &t, const std::vector<const Butterfly *> &bfs);
// n_x >= 0: run check_program (below) on the final tiles first
void upload_program(Program &prog, PackSink &pk, hipStream_t st, bool log = true,
                    int64_t n_x = -1, int64_t arena_count = -1);
// Host check of a packed program before it can reach a kernel: every tile's pairs read
// inside their input buffer (X: n_x rows, T: t_rows) and inside the factor arena
// (arena_count complex values; < 0 skips), and its row map writes inside the output.
// E_ARG on the first violation.
void check_program(const PackSink &pk, int64_t n_x, int64_t arena_count);
// Launches with fewer tiles than this get half-height tiles at upload (more workgroups).
// 512: with six waves per SIMD the split-BF16 kernel is 5-9% faster than with 1024 at
// 1-64 right-hand sides (the FP32 kernel is indifferent), and no faster with 0-384.
constexpr int64_t kRetileBelow = 512;
// Re-emit every launch's tiles, cutting those of launches with fewer than `below` tiles
// into tiles of at most `rows` rows (pairs offset to the rows, row maps clipped).
void retile(PackSink &pk, int64_t below, int rows);

}  // namespace hodbf
