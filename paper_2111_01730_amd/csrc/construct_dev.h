// Device side of the preconditioner construction: elementwise kernels and the device
// engine (construct.h) that runs Algorithm 1 / Algorithm 2 on the grouped-GEMM kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>

namespace hodbf {

class Engine;
struct Tree;

struct Seg;
struct Pair;
struct RowMap;

// Elementwise kernels on complex FP64 N x R multi-vectors (see construct.hip)
void launch_axpy_c128(double2 *y, const double2 *x, double ar, double ai, int64_t n, hipStream_t st);
void launch_keep_rows_c128(double2 *y, const uint8_t *keep, int64_t rows, int R, hipStream_t st);
void launch_fill_sketch_c128(double2 *x, const int32_t *slot, int64_t rows, int R, int64_t col0,
                             int k, uint64_t seed, hipStream_t st);
void launch_fill_unit_c128(double2 *x, const int32_t *col, int64_t rows, int R, hipStream_t st);
void launch_gather_rows_c128(const double2 *y, int R, const int32_t *rows, const int32_t *q0,
                             int64_t nent, int k, double2 *out, hipStream_t st);
// The grouped GEMM of the applies (same tiles, pairs and row maps) with FP64 vectors and
// accumulation over FP32-stored factors: OUT(rows) = beta OUT + sum A x.
void launch_grouped_f64(const Seg *segs, const Pair *pairs, const RowMap *rowmap, int64_t s0,
                        int64_t ns, const float2 *F, const double2 *X, const double2 *T,
                        double2 *OUT, int R, int beta, hipStream_t st);

// The device engine: multi-vectors in complex FP64 on the GPU (at most max_cols columns
// each), butterfly sets and dense blocks packed into grouped-GEMM programs (forward and
// transposed) run in FP64, everything on one stream.
std::unique_ptr<Engine> make_device_engine(const Tree *t, hipStream_t st, int max_cols);

}  // namespace hodbf
